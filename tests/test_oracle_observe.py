"""Pins of the oracle's observables on hand-built states.

The front z (section "Results and discussion": the centreline position of the
invading front, Fig. 2 and Eq. (1)), the grown solid thickness Delta e and
pore closure (Fig. 3: Delta e close to half the height means the pore has
closed) are read from the state by rules the paper states only in words; the
readings are:

* z: phi = rho1 / (rho1 + rho2) averaged over the centreline row(s) (rows
  y0 + W/2 - 1 and y0 + W/2 for even W, row y0 + (W-1)/2 for odd W); the
  first x from x_in with phi(x) >= 1/2 > phi(x+1), x + 1 < x_out, gives
  z = x + (phi(x) - 1/2) / (phi(x) - phi(x+1)) - x_in; z = 0 when
  phi(x_in) < 1/2; a solid centreline node met first gives z = its x - x_in;
  no crossing gives z = L = x_out - x_in (breakthrough).
* Delta e: per capillary column, d_b = consecutive solid nodes upward from
  row y0, d_t = the same downward from row y0 + W - 1; the column counts
  max(d_b, d_t), or W/2 when it is closed (d_b = W); Delta e is the largest.
* closure step: the step at which the first column closed, i.e. the minimum
  over closed columns of the latest step at which one of its nodes turned
  solid (0 for solid from the start).

Every expected value below is worked out in the test from these rules and
from the closed form of an isolated reacting node (C(n) = C0 (1 - 4 k_r)^n,
m(n) = C0 - C(n)), never read from the oracle.  The states are built so that
plausible slips give a different number: rows other than the centreline
carry other phases, the centreline rows carry different total densities (a
ratio of sums or rho1 alone would differ from the mean of phi), and the
event steps of the nodes in a column differ (a minimum instead of a maximum
would differ).
"""

import math

import numpy as np
import pytest

W9 = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)


class P:
    """Parameters for a hand-built state (no forces: the state stays at rest
    unless a node reacts)."""

    def __init__(self, nx, ny, **kw):
        self.nx, self.ny = nx, ny
        self.tau, self.G, self.G_ads1, self.G_ads2 = 1.0, 0.0, 0.0, 0.0
        self.tau_g, self.k_r, self.threshold = 0.0, 0.0, 1.0
        self.accel_x = self.accel_y = 0.0
        self.x_in = self.x_out = self.y0 = self.W = 0
        for k, v in kw.items():
            setattr(self, k, v)

    def replace(self, **kw):
        q = P(self.nx, self.ny)
        q.__dict__.update(self.__dict__)
        q.__dict__.update(kw)
        return q


def slit(nx, ny, W, y0, x_in, x_out):
    """Solid blocks above and below channel rows y0..y0+W-1 for
    x_in <= x < x_out; reservoirs fluid."""
    s = np.zeros((ny, nx), np.uint8)
    for y in range(ny):
        if not (y0 <= y < y0 + W):
            s[y, x_in:x_out] = 1
    return s


def phase_fields(solid, phi, total):
    """Densities with wetting fraction phi and total density `total` (arrays
    or scalars), zero at solids."""
    phi = np.broadcast_to(phi, solid.shape)
    total = np.broadcast_to(total, solid.shape)
    r1 = np.where(solid != 0, 0.0, phi * total)
    r2 = np.where(solid != 0, 0.0, (1.0 - phi) * total)
    return r1, r2


# --------------------------------------------------------------------------
# Front z: hand states (params, solid, rho1, rho2, expected z)
# --------------------------------------------------------------------------
def front_even_width():
    """W = 6, centre rows 5 and 6.  phi = 1 up to x = 16; at x = 17 rows 5/6
    hold 0.9/0.7 (mean 0.8), at x = 18 0.4/0.2 (mean 0.3), then 0.  The other
    channel rows are non-wetting everywhere.  Totals 1.0 (row 5) and 0.6
    (row 6): the ratio of summed densities would give 0.825 at x = 17.
    z = 17 + (0.8 - 0.5)/(0.8 - 0.3) - 10 = 7.6."""
    nx, ny, W, y0, xi, xo = 40, 12, 6, 3, 10, 32
    s = slit(nx, ny, W, y0, xi, xo)
    phi = np.zeros((ny, nx))
    tot = np.ones((ny, nx))
    phi[5, :17] = phi[6, :17] = 1.0
    phi[5, 17], phi[6, 17] = 0.9, 0.7
    phi[5, 18], phi[6, 18] = 0.4, 0.2
    tot[6, :] = 0.6
    r1, r2 = phase_fields(s, phi, tot)
    return P(nx, ny, W=W, y0=y0, x_in=xi, x_out=xo), s, r1, r2, 7.6


def front_odd_width():
    """W = 5, centre row 5 alone (rows 4 and 6 carry phi = 1 beyond the
    crossing).  phi(20) = 0.55, phi(21) = 0.05: z = 20 + 0.05/0.5 - 10 = 10.1."""
    nx, ny, W, y0, xi, xo = 40, 11, 5, 3, 10, 32
    s = slit(nx, ny, W, y0, xi, xo)
    phi = np.zeros((ny, nx))
    phi[5, :20] = 1.0
    phi[5, 20], phi[5, 21] = 0.55, 0.05
    phi[4, :30] = phi[6, :30] = 1.0
    r1, r2 = phase_fields(s, phi, 1.0)
    return P(nx, ny, W=W, y0=y0, x_in=xi, x_out=xo), s, r1, r2, 10.1


def front_first_crossing():
    """Two crossings: phi falls from 0.75 to 0.25 between x = 13 and 14,
    recovers, and falls again at x = 25.  The first counts:
    z = 13 + 0.25/0.5 - 10 = 3.5."""
    nx, ny, W, y0, xi, xo = 40, 11, 5, 3, 10, 32
    s = slit(nx, ny, W, y0, xi, xo)
    phi = np.zeros((ny, nx))
    phi[5, :14] = 1.0
    phi[5, 13], phi[5, 14] = 0.75, 0.25
    phi[5, 15:26] = 1.0
    r1, r2 = phase_fields(s, phi, 1.0)
    return P(nx, ny, W=W, y0=y0, x_in=xi, x_out=xo), s, r1, r2, 3.5


def front_exact_half():
    """phi(x) = 1/2 exactly is on the wetting side (phi >= 1/2), phi(x+1) =
    1/2 is not a crossing (1/2 > phi fails).  phi = 1 up to 14, 0.5 at 15 and
    16, 0.1 at 17: the crossing is at x = 16, z = 16 + 0 - 10 = 6."""
    nx, ny, W, y0, xi, xo = 40, 11, 5, 3, 10, 32
    s = slit(nx, ny, W, y0, xi, xo)
    phi = np.zeros((ny, nx))
    phi[5, :15] = 1.0
    phi[5, 15] = phi[5, 16] = 0.5
    phi[5, 17] = 0.1
    r1, r2 = phase_fields(s, phi, 1.0)
    return P(nx, ny, W=W, y0=y0, x_in=xi, x_out=xo), s, r1, r2, 6.0


def front_blocked():
    """Even W: a solid node in one of the two centreline rows at x = 19,
    before the crossing at 24: blocked, z = 19 - 10 = 9."""
    nx, ny, W, y0, xi, xo = 40, 12, 6, 3, 10, 32
    s = slit(nx, ny, W, y0, xi, xo)
    s[6, 19] = 1
    phi = np.zeros((ny, nx))
    phi[3:9, :24] = 1.0
    phi[3:9, 24] = 0.6
    r1, r2 = phase_fields(s, phi, 1.0)
    return P(nx, ny, W=W, y0=y0, x_in=xi, x_out=xo), s, r1, r2, 9.0


def front_solid_after_crossing():
    """A solid centreline node beyond the crossing does not matter:
    crossing 0.9 -> 0.1 at x = 15, solid at 25: z = 15 + 0.4/0.8 - 10 = 5.5."""
    nx, ny, W, y0, xi, xo = 40, 11, 5, 3, 10, 32
    s = slit(nx, ny, W, y0, xi, xo)
    s[5, 25] = 1
    phi = np.zeros((ny, nx))
    phi[5, :15] = 1.0
    phi[5, 15], phi[5, 16] = 0.9, 0.1
    r1, r2 = phase_fields(s, phi, 1.0)
    return P(nx, ny, W=W, y0=y0, x_in=xi, x_out=xo), s, r1, r2, 5.5


def front_not_entered():
    """phi(x_in) < 1/2: z = 0, although a crossing follows further in."""
    nx, ny, W, y0, xi, xo = 40, 11, 5, 3, 10, 32
    s = slit(nx, ny, W, y0, xi, xo)
    phi = np.zeros((ny, nx))
    phi[5, :10] = 1.0
    phi[5, 10] = 0.45
    phi[5, 11:20] = 1.0
    r1, r2 = phase_fields(s, phi, 1.0)
    return P(nx, ny, W=W, y0=y0, x_in=xi, x_out=xo), s, r1, r2, 0.0


def front_breakthrough():
    """phi >= 1/2 on every capillary column; the drop to 0 between x_out - 1
    and x_out lies outside the scanned range: z = L = 22."""
    nx, ny, W, y0, xi, xo = 40, 11, 5, 3, 10, 32
    s = slit(nx, ny, W, y0, xi, xo)
    phi = np.zeros((ny, nx))
    phi[:, :32] = 1.0
    phi[5, 31] = 0.6
    r1, r2 = phase_fields(s, phi, 1.0)
    return P(nx, ny, W=W, y0=y0, x_in=xi, x_out=xo), s, r1, r2, 22.0


FRONTS = {"even width": front_even_width, "odd width": front_odd_width,
          "first crossing": front_first_crossing, "exact half": front_exact_half,
          "blocked": front_blocked, "solid after crossing": front_solid_after_crossing,
          "not entered": front_not_entered, "breakthrough": front_breakthrough}


@pytest.mark.parametrize("name", list(FRONTS))
def test_front_position(oracle_mod, name):
    p, s, r1, r2, z = FRONTS[name]()
    o = oracle_mod.Oracle(p, s, r1, r2)
    got = o.observe()["front_z"]
    assert got == pytest.approx(z, abs=1e-12), (name, got, z)


def test_front_nan_without_capillary(oracle_mod):
    p, s, r1, r2, _ = front_odd_width()
    o = oracle_mod.Oracle(p.replace(W=0), s, r1, r2)
    assert math.isnan(o.observe()["front_z"])


def test_front_moves_with_the_interface(oracle_mod):
    """Shifting the phase pattern by one column shifts z by exactly one."""
    p, s, r1, r2, z = front_odd_width()
    o = oracle_mod.Oracle(p, s, np.roll(r1, 3, axis=1), np.roll(r2, 3, axis=1))
    assert o.observe()["front_z"] == pytest.approx(z + 3, abs=1e-12)


# --------------------------------------------------------------------------
# Delta e on fixed masks
# --------------------------------------------------------------------------
def test_delta_e_bumps(oracle_mod):
    """W = 9 between rows 2 and 10.  Column 12: three solid nodes on the
    lower wall (d_b = 3).  Column 15: two on the upper wall (d_t = 2).
    Column 18: a solid node one row off the wall (not consecutive: 0).
    Column 20: lower wall rows 2 and 4 (d_b = 1).  Column 24: d_b = 2 and
    d_t = 6 with one fluid node between, open: max = 6 > W/2 = 4.5."""
    nx, ny, W, y0, xi, xo = 40, 13, 9, 2, 10, 30
    s = slit(nx, ny, W, y0, xi, xo)
    s[2:5, 12] = 1
    s[9:11, 15] = 1
    s[3, 18] = 1
    s[2, 20] = s[4, 20] = 1
    p = P(nx, ny, W=W, y0=y0, x_in=xi, x_out=xo)
    r1, r2 = phase_fields(s, 0.0, 1.0)
    o = oracle_mod.Oracle(p, s, r1, r2)
    ob = o.observe()
    assert ob["delta_e"] == 3.0 and ob["closure_step"] == -1
    s2 = s.copy()
    s2[2:4, 24] = 1
    s2[5:11, 24] = 1
    r1, r2 = phase_fields(s2, 0.0, 1.0)
    ob = oracle_mod.Oracle(p, s2, r1, r2).observe()
    assert ob["delta_e"] == 6.0 and ob["closure_step"] == -1
    # outside the capillary section solid nodes do not count
    s3 = s.copy()
    s3[2:10, 5] = 1
    s3[2:10, 31] = 1
    r1, r2 = phase_fields(s3, 0.0, 1.0)
    assert oracle_mod.Oracle(p, s3, r1, r2).observe()["delta_e"] == 3.0


def test_delta_e_closed_column_is_half_width(oracle_mod):
    """A column solid across the whole channel from the start counts W/2
    (here 3.5 for W = 7, below the 5-node bump elsewhere, which wins) and
    closes the pore at step 0."""
    nx, ny, W, y0, xi, xo = 40, 11, 7, 2, 10, 30
    s = slit(nx, ny, W, y0, xi, xo)
    s[2:9, 22] = 1
    p = P(nx, ny, W=W, y0=y0, x_in=xi, x_out=xo)
    r1, r2 = phase_fields(s, 0.0, 1.0)
    ob = oracle_mod.Oracle(p, s, r1, r2).observe()
    assert ob["delta_e"] == 3.5 and ob["closure_step"] == 0
    s[4:9, 14] = 1
    r1, r2 = phase_fields(s, 0.0, 1.0)
    ob = oracle_mod.Oracle(p, s, r1, r2).observe()
    assert ob["delta_e"] == 5.0 and ob["closure_step"] == 0


# --------------------------------------------------------------------------
# Closure step from reacting pockets
# --------------------------------------------------------------------------
K_R = 0.01
POCKETS = {(7, 2): 2.0, (7, 7): 1.5, (12, 2): 1.8, (12, 7): 1.8}


def event_step(c0, k_r=K_R, threshold=1.0):
    """First n with m(n) = c0 (1 - (1 - 4 k_r)^n) > threshold (isolated node,
    phi = 1, four solid axis neighbours)."""
    n = 0
    while c0 * (1.0 - (1.0 - 4.0 * k_r) ** n) <= threshold:
        n += 1
    return n


def pocket_state():
    """W = 6 between rows 2 and 7, capillary x in [3, 17).  Columns 7 and 12
    each hold two isolated one-node pockets, on the lower (row 2) and upper
    (row 7) wall, with the four nodes between them solid; the columns either
    side are solid at rows 2, 3, 6 and 7, so every pocket has eight solid
    neighbours and decays by the closed form.  Pocket concentrations 2.0 and
    1.5 (column 7) and 1.8 and 1.8 (column 12); everything else is
    non-wetting fluid without solute, at rest."""
    nx, ny, W, y0, xi, xo = 20, 10, 6, 2, 3, 17
    s = slit(nx, ny, W, y0, xi, xo)
    for xc in (7, 12):
        s[3:7, xc] = 1
        for xs in (xc - 1, xc + 1):
            s[[2, 3, 6, 7], xs] = 1
    phi = np.zeros((ny, nx))
    c = np.zeros((ny, nx))
    for (x, y), c0 in POCKETS.items():
        phi[y, x] = 1.0
        c[y, x] = c0
    r1, r2 = phase_fields(s, phi, 1.0)
    p = P(nx, ny, W=W, y0=y0, x_in=xi, x_out=xo, tau_g=0.65, k_r=K_R, threshold=1.0)
    return p, s, r1, r2, c


def pocket_expectations():
    """(step, delta_e, closure_step) worked out by hand: column 7 turns its
    lower pocket solid at event_step(2.0) = 17 (d_b becomes 5: rows 2..6),
    closes at event_step(1.5) = 27; column 12 closes when both pockets turn
    solid at event_step(1.8) = 20.  The side columns always give 2."""
    a, b, c = event_step(2.0), event_step(1.5), event_step(1.8)
    assert (a, b, c) == (17, 27, 20)
    rows = []
    for n in (1, a - 1, a, c - 1, c, b - 1, b, b + 5):
        col7 = 3.0 if n >= b else (5.0 if n >= a else 0.0)
        col12 = 3.0 if n >= c else 0.0
        de = max(2.0, col7, col12)
        closure = min([t for t in (c if n >= c else None, b if n >= b else None)
                       if t is not None], default=-1)
        rows.append((n, de, closure))
    return rows


def test_closure_step_from_pockets(oracle_mod):
    p, s, r1, r2, c = pocket_state()
    o = oracle_mod.Oracle(p, s, r1, r2, c)
    ob = o.observe()
    assert ob["delta_e"] == 2.0 and ob["closure_step"] == -1
    for n, de, closure in pocket_expectations():
        o.step(n - o.steps)
        ob = o.observe()
        assert (ob["delta_e"], ob["closure_step"]) == (de, closure), (n, ob["delta_e"],
                                                                      ob["closure_step"])
    ev = sorted((int(e["x"]), int(e["y"]), int(e["step"])) for e in o.events())
    assert ev == sorted((x, y, event_step(c0)) for (x, y), c0 in POCKETS.items())
