"""The largest lattice the library accepts, on the GPU.

Element offsets inside the kernels are 32-bit: the 23 population planes of a
lattice must stay below 2^31 elements, and the moment step's buffer
descriptors carry byte offsets up to 24 * P.  The lattice here sits just under
that limit (23 P = 2,147,188,736).

The lattice is periodic in x and y (Sec. 2, periodic streaming) and the
per-node arithmetic does not depend on the launch shape, so a small reactive
capillary tiled m x n times must evolve into bit-exact periodic copies of the
small run: every field and every growth event.  The small run itself is held
to the oracle by the parity tests; here the full-size lattice is held to the
small run, in both step schemes, in the launch shapes the benchmark uses.
"""

import numpy as np
import pytest

import parity as PT
from paper_1309_6726_amd import inputs

pytestmark = pytest.mark.gpu

NX_S, NY_S = 256, 32          # small periodic cell: capillary W = 20
REP_X, REP_Y = 37, 308        # 9472 x 9856 = 93,356,032 nodes
STEPS = 700


@pytest.fixture(scope="module")
def lbm():
    from paper_1309_6726_amd import lbm as L
    L.lib()
    return L


def _small():
    return inputs.capillary_problem(NX_S, NY_S, 20, seed=5, k_r=0.01, threshold=0.4, D=0.05)


def _tiled(prob):
    p = prob.params.replace(nx=NX_S * REP_X, ny=NY_S * REP_Y)
    t = lambda a: np.tile(a, (REP_Y, REP_X))
    return inputs.Problem(p, t(prob.solid), t(prob.rho1), t(prob.rho2), t(prob.conc))


@pytest.mark.parametrize("scheme,tile,hint", [("moments", (64, 9), 0), ("moments", (64, 12), 1),
                                              ("populations", (256, 40), 1)])
def test_max_lattice_is_periodic_copies_of_small(lbm, scheme, tile, hint):
    small = _small()
    PT.say(f"[max size] small {NX_S}x{NY_S} {scheme} {tile} hint {hint}: {STEPS} steps")
    s = lbm.Sim.from_problem(small, tile=tile, scheme=scheme)
    s.set_load_hint(hint)
    s.step(STEPS)
    fs = s.fields()
    ev_s = s.events()
    s.close()
    assert len(ev_s) > 0

    big = _tiled(small)
    nx, ny = big.params.nx, big.params.ny
    PT.say(f"[max size] tiled {nx}x{ny} ({nx * ny} nodes) {scheme} {tile}: {STEPS} steps")
    b = lbm.Sim.from_problem(big, tile=tile, scheme=scheme)
    b.set_load_hint(hint)
    del big
    b.step(STEPS)
    for name, small_field in fs.items():
        f = b.fields(names=(name,))[name]
        cells = f.reshape(REP_Y, NY_S, REP_X, NX_S)
        same = cells == small_field[None, :, None, :]
        assert same.all(), (scheme, name, int((~same).sum()))
        del f, cells, same

    # every event of the small run, once per copy, at the same step
    ev_b = b.events()
    b.close()
    assert len(ev_b) == len(ev_s) * REP_X * REP_Y
    ox = (np.arange(REP_X) * NX_S)[None, :, None]
    oy = (np.arange(REP_Y) * NY_S)[:, None, None]
    want_x = (ev_s["x"][None, None, :] + ox + 0 * oy).ravel()
    want_y = (ev_s["y"][None, None, :] + oy + 0 * ox).ravel()
    want_t = np.broadcast_to(ev_s["step"][None, None, :], (REP_Y, REP_X, len(ev_s))).ravel()
    want = np.sort(np.rec.fromarrays([want_y, want_x, want_t], names="y,x,step"), order=["y", "x", "step"])
    got = np.sort(np.rec.fromarrays([ev_b["y"], ev_b["x"], ev_b["step"]], names="y,x,step"),
                  order=["y", "x", "step"])
    assert np.array_equal(got, want)
