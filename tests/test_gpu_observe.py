"""The library's observables on the hand-built states of the oracle's
observable pins (front z, Delta e and pore closure; section "Results and
discussion", Figs. 2-3), through the C ABI.

The expected values are the ones worked out by hand in test_oracle_observe;
the GPU stores densities in FP32, so the front may differ from the hand value
by the FP32 rounding of phi (the bound below is 1e-5 lattice units), while
Delta e, the closure step and the growth events are integer results and must
be equal.
"""

import numpy as np
import pytest

import parity as PT
import test_oracle_observe as H

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lbm():
    from paper_1309_6726_amd import lbm as L
    L.lib()
    return L


class _Prob:
    def __init__(self, p, solid, r1, r2, c):
        self.params, self.solid, self.rho1, self.rho2, self.conc = p, solid, r1, r2, c


@pytest.mark.parametrize("name", list(H.FRONTS))
def test_front_hand_states(lbm, name):
    p, s, r1, r2, z = H.FRONTS[name]()
    PT.say(f"[observe front] {name}: {p.nx}x{p.ny} W={p.W}, expected z={z}")
    sim = lbm.Sim(p, s, r1, r2)
    got = sim.observe()["front_z"]
    assert abs(got - z) <= 1e-5, (name, got, z)


def test_delta_e_hand_masks(lbm):
    nx, ny, W, y0, xi, xo = 40, 13, 9, 2, 10, 30
    s = H.slit(nx, ny, W, y0, xi, xo)
    s[2:5, 12] = 1
    s[9:11, 15] = 1
    s[3, 18] = 1
    s[2, 20] = s[4, 20] = 1
    p = H.P(nx, ny, W=W, y0=y0, x_in=xi, x_out=xo)
    PT.say("[observe delta_e] bumps on a 40x13 slit")
    r1, r2 = H.phase_fields(s, 0.0, 1.0)
    ob = lbm.Sim(p, s, r1, r2).observe()
    assert ob["delta_e"] == 3.0 and ob["closure_step"] == -1
    s[2:4, 24] = 1
    s[5:11, 24] = 1
    r1, r2 = H.phase_fields(s, 0.0, 1.0)
    ob = lbm.Sim(p, s, r1, r2).observe()
    assert ob["delta_e"] == 6.0 and ob["closure_step"] == -1


@pytest.mark.parametrize("scheme", ["moments", "populations"])
def test_closure_step_from_pockets(lbm, scheme):
    """Isolated reacting pockets whose event steps follow from the closed
    form: Delta e and the closure step at every hand-computed step."""
    p, s, r1, r2, c = H.pocket_state()
    PT.say(f"[observe closure] pockets, {scheme}")
    sim = lbm.Sim(p, s, r1, r2, c, scheme=scheme)
    done = 0
    for n, de, closure in H.pocket_expectations():
        sim.step(n - done)
        done = n
        ob = sim.observe()
        assert (ob["delta_e"], ob["closure_step"]) == (de, closure), (n, ob["delta_e"],
                                                                      ob["closure_step"])
    ev = sorted(PT.event_set(sim.events()))
    assert ev == sorted((x, y, H.event_step(c0)) for (x, y), c0 in H.POCKETS.items())


def test_closure_step_batched(lbm):
    """The same pockets as one instance of a batch beside a reactive
    capillary: the batched observer gives the hand values too."""
    from paper_1309_6726_amd import inputs
    p, s, r1, r2, c = H.pocket_state()
    other = inputs.capillary_problem(96, 24, 10, seed=2, k_r=0.02, threshold=0.3, D=0.05)
    other.params = other.params.replace(G=0.0)  # a batch shares G
    PT.say("[observe closure] pockets in a batch")
    b = lbm.Batch([_Prob(p, s, r1, r2, c), other])
    done = 0
    for n, de, closure in H.pocket_expectations():
        b.step(n - done)
        done = n
        ob = b.observe(0)
        assert (ob["delta_e"], ob["closure_step"]) == (de, closure), (n, ob)
    b.close()
