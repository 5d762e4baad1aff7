"""GPU (HIP: FP32 state, FP64 arithmetic) vs FP64 oracle parity through the C ABI.

Every test prints the case it runs before touching the GPU.
"""

import numpy as np
import pytest

import parity as PT
from paper_1309_6726_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lbm():
    from paper_1309_6726_amd import lbm as L
    L.lib()
    return L


def _fields_cmp(sim, orc, where, **kw):
    gf = sim.fields()
    of = orc.fields()
    return PT.compare_fields(gf, of, where=where, **kw)


# ---------------------------------------------------------------------------
def test_config0_parity_2000_steps(lbm, oracle_mod):
    """256x32 capillary, W=20, no reaction: densities, velocity, masses and
    the front every 200 steps up to 2000."""
    prob = inputs.config0(seed=0)
    PT.say(f"[cfg0] {prob.name}: 2000 steps")
    sim = lbm.Sim.from_problem(prob)
    orc = oracle_mod.Oracle.from_problem(prob)
    o0 = orc.observe()
    for n in range(200, 2001, 200):
        sim.step(200)
        orc.step(200)
        go, oo = sim.observe(), orc.observe()
        assert go["step"] == oo["step"] == n
        assert abs(go["front_z"] - oo["front_z"]) <= PT.Z_TOL, (n, go["front_z"], oo["front_z"])
        for s in range(2):
            assert abs(go["mass"][s] - o0["mass"][s]) <= PT.MASS_TOL * o0["mass"][s]
        if n in (1000, 2000):
            d = _fields_cmp(sim, orc, f"cfg0 step {n}")
            PT.say(f"  step {n}: z gpu {go['front_z']:.4f} cpu {oo['front_z']:.4f}; {d}")
    assert oo["front_z"] > 5.0  # the wetting fluid has entered the capillary


@pytest.mark.parametrize("seed", [1, 2])
def test_config0_other_seeds(lbm, oracle_mod, seed):
    prob = inputs.config0(seed=seed)
    PT.say(f"[cfg0 seed {seed}] 1000 steps")
    sim = lbm.Sim.from_problem(prob)
    orc = oracle_mod.Oracle.from_problem(prob)
    sim.step(1000)
    orc.step(1000)
    _fields_cmp(sim, orc, f"cfg0 seed {seed}")


def _random_state(nx, ny, seed, solid_frac=0.25, m_hi=0.5):
    rng = np.random.default_rng(seed)
    solid = (rng.uniform(size=(ny, nx)) < solid_frac).astype(np.uint8)
    # populations near a two-phase equilibrium, perturbed (non-equilibrium start)
    phase = rng.uniform(size=(ny, nx)) < 0.5
    r1 = np.where(phase, 1.0, 0.05)
    r2 = np.where(phase, 0.05, 1.0)
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    f = np.concatenate([w[:, None, None] * r1, w[:, None, None] * r2])
    f = f * rng.uniform(0.9, 1.1, f.shape)
    g = np.array([1 / 3] + [1 / 6] * 4)[:, None, None] * rng.uniform(0, 1, (ny, nx))
    m = rng.uniform(0, m_hi, (ny, nx))
    f = np.where(solid[None] != 0, 0.0, f).astype(np.float32).astype(np.float64)
    g = np.where(solid[None] != 0, 0.0, g).astype(np.float32).astype(np.float64)
    m = np.where(solid != 0, 0.0, m)
    return solid, f, g, m


def _random_state_run(lbm, oracle_mod, nx, ny, tile, tau, **variant):
    solid, f, g, m = _random_state(nx, ny, seed=nx * 1000 + ny)
    if variant.get("solute_q") == 4:
        g[0] = 0.0  # D2Q4: no rest link
    # prime a few wall-adjacent nodes to grow within the run
    walls = sum(np.roll(solid, s, axis=a) for s in (1, -1) for a in (0, 1))
    cand = np.argwhere((solid == 0) & (walls > 0))
    for k in range(min(5, len(cand))):
        m[tuple(cand[k * len(cand) // 5])] = 0.9985 + 0.0001 * k
    p = inputs.Params(nx=nx, ny=ny, tau=tau, G=1.6, G_ads1=-0.33, G_ads2=0.33, tau_g=0.65,
                      k_r=0.01, threshold=1.0, accel_x=2e-5, accel_y=-1e-5, **variant)
    sim = lbm.Sim(p, solid, np.where(solid, 0.0, 1.0), np.where(solid, 0.0, 1.0),
                  np.zeros((ny, nx)), tile=tile)
    sim.load_state(f, solid, g, m)
    orc = oracle_mod.Oracle(p, solid, f=f, g=g, m=m)
    for n in (1, 5, 30):
        sim.step(n - orc.steps)
        orc.step(n - orc.steps)
        _fields_cmp(sim, orc, f"random {nx}x{ny} step {n}", rho_tol=2e-5, u_tol=2e-5,
                    conc_tol=2e-5, m_tol=1e-6)
        assert PT.event_set(sim.events()) == PT.event_set(orc.events())
    assert len(orc.events()) >= 1
    go, oo = sim.observe(), orc.observe()
    for k in ("solute", "precipitate", "solute_removed"):
        assert abs(go[k] - oo[k]) <= 1e-5 * max(1.0, abs(oo[k])), k
    for s in range(2):
        assert abs(go["mass_removed"][s] - oo["mass_removed"][s]) <= 1e-5 * max(1.0, oo["mass_removed"][s])
    assert go["n_solid"] == oo["n_solid"] and go["n_events"] == oo["n_events"]


@pytest.mark.parametrize("tau", [0.9, 1.0])
@pytest.mark.parametrize("nx,ny,tile", [(8, 8, (64, 4)), (37, 23, (64, 8)), (300, 19, (128, 16)),
                                        (509, 40, (256, 32))])
def test_random_state_all_terms(lbm, oracle_mod, nx, ny, tile, tau):
    """Random non-equilibrium two-phase states with random walls and
    precipitate, every term on (forces, adhesion, body force, solute,
    reaction, growth), ragged tiles: 30 steps, fields and events.  At
    tau = 1 the first step reads the loaded populations and stores moments;
    the later steps rebuild the populations from moments (growth bookings
    and mask folds included)."""
    PT.say(f"[random state] {nx}x{ny} tile {tile} tau {tau}")
    _random_state_run(lbm, oracle_mod, nx, ny, tile, tau)


VARIANTS = {"saturation": dict(c_eq=0.3), "held source": dict(hold_x=7, c_hold=0.7),
            "d2q4": dict(solute_q=4), "all": dict(c_eq=0.2, hold_x=5, c_hold=0.9, solute_q=4)}


@pytest.mark.parametrize("tau", [0.9, 1.0])
@pytest.mark.parametrize("variant", list(VARIANTS))
@pytest.mark.parametrize("nx,ny,tile", [(37, 23, (64, 8)), (300, 19, (128, 16))])
def test_reaction_variants(lbm, oracle_mod, nx, ny, tile, variant, tau):
    """Saturation concentration, held source and the D2Q4 solute lattice on
    random states (every other term on), against the oracle, both schemes."""
    PT.say(f"[variant {variant}] {nx}x{ny} tile {tile} tau {tau}")
    _random_state_run(lbm, oracle_mod, nx, ny, tile, tau, **VARIANTS[variant])


def test_d2q4_checkpoint_rejects_rest_population(lbm):
    p = inputs.Params(nx=16, ny=8, tau_g=0.7, solute_q=4)
    solid = np.zeros((8, 16), np.uint8)
    sim = lbm.Sim(p, solid, np.ones((8, 16)), np.zeros((8, 16)), np.ones((8, 16)))
    f = np.zeros((18, 8, 16))
    f[0] = 1.0
    g = np.zeros((5, 8, 16))
    g[1:] = 0.25
    sim.load_state(f, solid, g)
    g[0, 3, 3] = 0.1
    with pytest.raises(lbm.LbmError) as e:
        sim.load_state(f, solid, g)
    assert e.value.status == lbm.LBM_EINVAL


@pytest.mark.timeout(900)
def test_config1_events_exact_50k_steps(lbm, oracle_mod):
    """1024x64 reactive capillary (W=48, D=0.05, k_r=1e-3, threshold 1) over
    its full 50,000 steps: growth events compared exactly in windows of 1000
    steps (no difference tolerated), fields within tolerance, the front, Delta
    e, the closure step and both ledgers at every window boundary."""
    prob = inputs.config1(seed=0)
    nsteps = 50_000
    PT.say(f"[cfg1] {prob.name}: {nsteps} steps in windows of 1000")
    sim = lbm.Sim.from_problem(prob)
    orc = oracle_mod.Oracle.from_problem(prob)
    o0 = orc.observe()
    MASS_REL = 1e-6

    def check(step, sim, orc):
        go, oo = sim.observe(), orc.observe()
        assert abs(go["front_z"] - oo["front_z"]) <= PT.Z_TOL, (step, go["front_z"], oo["front_z"])
        assert go["delta_e"] == oo["delta_e"] and go["closure_step"] == oo["closure_step"]
        assert go["n_solid"] == oo["n_solid"]
        tot = go["solute"] + go["precipitate"] + go["solute_removed"]
        assert abs(tot - o0["solute"]) <= MASS_REL * o0["solute"]
        for s in range(2):
            assert abs(go["mass"][s] + go["mass_removed"][s] - o0["mass"][s]) <= MASS_REL * o0["mass"][s]
        _fields_cmp(sim, orc, f"cfg1 step {step}")

    nev, _, dm, orc = PT.run_windows(sim, orc, nsteps, 1000, field_check=check)
    oo = orc.observe()
    PT.say(f"  cfg1: {nev} growth events identical over {nsteps} steps, max |dm| {dm:.2e}, "
           f"delta_e {oo['delta_e']}, closure step {oo['closure_step']}")
    assert nev > 1000


@pytest.mark.parametrize("scheme", ["moments", "populations"])
def test_tile_shapes_bitwise_identical(lbm, scheme):
    """The launch shape changes no result bit (reactive run with events)."""
    prob = inputs.capillary_problem(300, 40, 20, seed=5, k_r=0.01, threshold=0.4, D=0.05)
    ref = None
    for tile in [(64, 4), (128, 16), (256, 7), (64, 64), (256, 40)]:
        PT.say(f"[tiles] {scheme} {tile}")
        sim = lbm.Sim.from_problem(prob, tile=tile, scheme=scheme)
        sim.step(700)
        blob = sim.save()
        ev = sorted(PT.event_set(sim.events()))
        if ref is None:
            ref = (blob, ev)
            assert len(ev) > 0
        else:
            # event order inside the log may differ; the state must not
            assert ev == ref[1]
            hdr = 40
            N = 300 * 40
            body = 18 * N * 4 + 5 * N * 4 + N + N * 8 + N * 4 + 3 * N * 4
            assert blob[:hdr + body] == ref[0][:hdr + body], tile


@pytest.mark.parametrize("scheme", ["moments", "populations"])
def test_tile_shapes_bitwise_sweep_geometry(lbm, scheme):
    """Regression: a sweep instance (narrow throat, solute front with tiny
    far-field concentrations) over 600 steps.  Row segments of different
    heights put different rows in the peeled first iterations of the row
    loop; fusion of multiply-adds chosen per copy of the loop body once made
    the last bit of a few concentrations depend on the tile height."""
    rows = inputs.sweep_params(11, 5)
    W, nx, k, th, thr = rows[0]
    prob = inputs.sweep_problem((W, 256 + (int(nx) % 300), 0.005, th, 0.3), instance=0)
    ref = None
    for tile in [(64, 16), (64, 24), (64, 12), (128, 16)]:
        PT.say(f"[tiles sweep geometry] {scheme} {tile}")
        sim = lbm.Sim.from_problem(prob, tile=tile, scheme=scheme)
        sim.step(600)
        blob = sim.save()
        ev = sorted(PT.event_set(sim.events()))
        # the event log ends the blob; its order may differ, its content not
        n_ev = int(np.frombuffer(blob[32:40], dtype=np.int64)[0])
        state = blob[:len(blob) - n_ev * lbm.EVENT_DTYPE.itemsize]
        if ref is None:
            ref = (state, ev)
        else:
            assert ev == ref[1], tile
            assert state == ref[0], tile


# The launch shapes lbm_autotune times: TX 64/128/256 (64 only in the moment
# step), SY from this list (heights beyond 2 ny skipped), both load hints.
AUTOTUNE_SY = (6, 8, 9, 10, 12, 16, 20, 24, 28, 32, 40, 48, 64, 96, 128)


@pytest.mark.parametrize("scheme", ["moments", "populations"])
def test_every_autotune_candidate_bitwise(lbm, scheme):
    """Whatever shape and load hint the autotuner picks, the run is the same
    bit for bit (state and growth events), and a repeat of one shape too."""
    prob = inputs.capillary_problem(300, 40, 20, seed=7, k_r=0.01, threshold=0.4, D=0.05)
    txs = (64,) if scheme == "moments" else (64, 128, 256)
    shapes = [(tx, sy, nt) for nt in (0, 1) for tx in txs for sy in AUTOTUNE_SY if sy <= 2 * 40]
    shapes.append(shapes[0])  # a repeat
    PT.say(f"[autotune candidates] {scheme}: {len(shapes)} runs of 300 steps")
    ref = None
    for tx, sy, nt in shapes:
        sim = lbm.Sim.from_problem(prob, tile=(tx, sy), scheme=scheme)
        sim.set_load_hint(nt)
        sim.step(300)
        blob = sim.save()
        n_ev = int(np.frombuffer(blob[32:40], dtype=np.int64)[0])
        state = blob[:len(blob) - n_ev * lbm.EVENT_DTYPE.itemsize]
        ev = sorted(PT.event_set(sim.events()))
        sim.close()
        if ref is None:
            ref = (state, ev)
            assert len(ev) > 0
        else:
            assert ev == ref[1] and state == ref[0], (tx, sy, nt)


@pytest.mark.parametrize("scheme", ["moments", "populations"])
def test_load_hint_changes_no_bit(lbm, scheme):
    """The non-temporal load hint is a cache policy: same state and events."""
    prob = inputs.capillary_problem(300, 40, 20, seed=5, k_r=0.01, threshold=0.4, D=0.05)
    ref = None
    for nt in (0, 1):
        PT.say(f"[load hint] {scheme} nt={nt}")
        sim = lbm.Sim.from_problem(prob, tile=(64, 12), scheme=scheme)
        sim.set_load_hint(nt)
        sim.step(700)
        blob = sim.save()
        ev = sorted(PT.event_set(sim.events()))
        n_ev = int(np.frombuffer(blob[32:40], dtype=np.int64)[0])
        state = blob[:len(blob) - n_ev * lbm.EVENT_DTYPE.itemsize]
        if ref is None:
            ref = (state, ev)
            assert len(ev) > 0
        else:
            assert ev == ref[1] and state == ref[0], scheme


def test_schemes_agree(lbm, oracle_mod):
    """tau = 1: populations and moments between steps give the same run to
    FP32 rounding: fields, masses, fronts and the exact growth events."""
    prob = inputs.capillary_problem(300, 40, 20, seed=5, k_r=0.01, threshold=0.4, D=0.05)
    PT.say("[schemes] 300x40 reactive capillary, 1500 steps, populations vs moments")
    a = lbm.Sim.from_problem(prob, scheme="populations")
    b = lbm.Sim.from_problem(prob, scheme="moments")
    for n in (1, 2, 3, 500, 1500):
        a.step(n - a.observe()["step"])
        b.step(n - b.observe()["step"])
        fa, fb = a.fields(), b.fields()
        fb = dict(fb, m=fb["precip"])
        d = PT.compare_fields(fa, fb, m_tol=1e-6, where=f"schemes step {n}")
        oa, ob = a.observe(), b.observe()
        for s in range(2):
            assert abs(oa["mass"][s] - ob["mass"][s]) <= 1e-6 * oa["mass"][s]
        assert abs(oa["front_z"] - ob["front_z"]) <= PT.Z_TOL
        assert oa["n_solid"] == ob["n_solid"] and oa["closure_step"] == ob["closure_step"]
        assert PT.event_set(a.events()) == PT.event_set(b.events())
        PT.say(f"  step {n}: {d}")
    assert len(a.events()) > 0
    with pytest.raises(lbm.LbmError) as e:
        lbm.Sim(prob.params.replace(tau=0.9), prob.solid, prob.rho1, prob.rho2, prob.conc,
                scheme="moments")
    assert e.value.status == lbm.LBM_EINVAL


def test_checkpoint_resume_bitwise(lbm):
    prob = inputs.capillary_problem(256, 40, 24, seed=3, k_r=0.01, threshold=0.5, D=0.05)
    PT.say("[checkpoint] 400 + 400 vs 800 steps")
    a = lbm.Sim.from_problem(prob)
    a.step(400)
    blob = a.save()
    a.step(400)
    b = lbm.Sim.from_problem(prob)
    b.load(blob)
    b.step(400)
    # the event log order within a step may differ; the state and the event set may not
    hdr, N = 40, 256 * 40
    body = 18 * N * 4 + 5 * N * 4 + N + N * 8 + N * 4 + 3 * N * 4
    assert a.save()[:hdr + body] == b.save()[:hdr + body]
    assert PT.event_set(a.events()) == PT.event_set(b.events())
    assert len(a.events()) > 0
    fa, fb = a.fields(), b.fields()
    for k in fa:
        assert np.array_equal(fa[k], fb[k]), k
    assert a.observe() == b.observe()


@pytest.mark.timeout(900)
def test_config2_full_domain_1000_steps_and_first_events(lbm, oracle_mod):
    """2048x2048 porous preform, whole lattice, in the launch configuration
    the benchmark's autotuner picks for it on MI355X (moment step, 64x12
    tiles, non-temporal load hint), against the oracle on all host threads:
    every field at step 1000 (densities 1e-5, velocity 1e-6, concentration
    1e-5, precipitate 1e-6), masses and ledgers, and the growth events of the
    preform compared exactly through step 1300 (the first ones appear near
    step 770)."""
    prob = inputs.config2(seed=0)
    PT.say(f"[cfg2] {prob.name}: full domain, 1000 + 300 steps")
    sim = lbm.Sim.from_problem(prob, tile=(64, 12))
    sim.set_load_hint(1)
    orc = oracle_mod.Oracle.from_problem(prob)
    o0 = orc.observe()
    for n in (1000, 1300):
        sim.step(n - orc.steps)
        orc.step(n - orc.steps)
        go, oo = sim.observe(), orc.observe()
        d = _fields_cmp(sim, orc, f"cfg2 step {n}", m_tol=1e-6)
        for s in range(2):
            assert abs(go["mass"][s] + go["mass_removed"][s] - o0["mass"][s]) <= 1e-6 * o0["mass"][s]
            assert abs(go["mass"][s] - oo["mass"][s]) <= 1e-6 * oo["mass"][s]
        tot = go["solute"] + go["precipitate"] + go["solute_removed"]
        assert abs(tot - o0["solute"]) <= 1e-6 * o0["solute"]
        ge, oe = PT.event_set(sim.events()), PT.event_set(orc.events())
        assert ge == oe, (n, len(ge - oe), len(oe - ge))
        assert go["n_solid"] == oo["n_solid"]
        PT.say(f"  step {n}: {len(ge)} growth events identical; {d}")
    assert len(ge) >= 50


@pytest.mark.timeout(900)
def test_population_step_preform_full_domain(lbm, oracle_mod):
    """The population step (any tau) on the whole 2048x2048 preform at
    tau = 0.8, in its benchmark launch shape (256x6 tiles, non-temporal
    loads), against the oracle after 500 steps: every field, masses and
    ledgers within the parity tolerances."""
    prob = inputs.config2(seed=0)
    p = prob.params.replace(tau=0.8)
    PT.say(f"[population step] {prob.name} at tau 0.8: full domain, 500 steps")
    sim = lbm.Sim(p, prob.solid, prob.rho1, prob.rho2, prob.conc, tile=(256, 6))
    sim.set_load_hint(1)
    orc = oracle_mod.Oracle(p, prob.solid, prob.rho1, prob.rho2, prob.conc)
    o0 = orc.observe()
    sim.step(500)
    orc.step(500)
    go = sim.observe()
    d = _fields_cmp(sim, orc, "population step preform step 500", m_tol=1e-6)
    for c in range(2):
        assert abs(go["mass"][c] + go["mass_removed"][c] - o0["mass"][c]) <= 1e-6 * o0["mass"][c]
    tot = go["solute"] + go["precipitate"] + go["solute_removed"]
    assert abs(tot - o0["solute"]) <= 1e-6 * o0["solute"]
    PT.say(f"  {d}")


def test_edge_lattices(lbm, oracle_mod):
    """Smallest lattice, a lattice with no fluid, one without solid, a single
    component, no solute, ragged tiles."""
    cases = []
    p = inputs.Params(nx=3, ny=3, G=1.6, tau_g=0.65)
    cases.append(("3x3 fluid", p, np.zeros((3, 3), np.uint8)))
    p = inputs.Params(nx=5, ny=4, tau_g=0.65, k_r=0.01)
    cases.append(("all solid", p, np.ones((4, 5), np.uint8)))
    p = inputs.Params(nx=67, ny=5, G=0.0, G_ads1=0.0, G_ads2=0.0, accel_x=1e-5)
    s = np.zeros((5, 67), np.uint8)
    s[0] = 1
    cases.append(("single component channel", p, s))
    for name, p, solid in cases:
        PT.say(f"[edge] {name}")
        ny, nx = solid.shape
        r1 = np.where(solid, 0.0, 0.7)
        r2 = np.where(solid, 0.0, 0.0 if "single" in name else 0.2)
        c = np.where(solid, 0.0, 0.3) if p.tau_g > 0 else None
        sim = lbm.Sim(p, solid, r1, r2, c)
        orc = oracle_mod.Oracle(p, solid, r1, r2, c)
        sim.step(50)
        orc.step(50)
        go, oo = sim.observe(), orc.observe()
        assert go["n_solid"] == oo["n_solid"]
        if solid.all():
            assert go["mass"] == (0.0, 0.0)
            continue
        _fields_cmp(sim, orc, name)


def _degenerate(name, nx, ny):
    """Geometries at the edges of what the step meets: every fluid node with
    four solid axis neighbours, fluid nodes enclosed on all eight sides, a
    channel one node wide, and wall bumps that grow across the periodic seam."""
    s = np.zeros((ny, nx), np.uint8)
    yy, xx = np.mgrid[0:ny, 0:nx]
    if name == "checkerboard":
        s[(xx + yy) % 2 == 1] = 1
    elif name == "isolated nodes":
        s[:] = 1
        s[1::3, 1::3] = 0
    elif name == "one-wide channel":
        s[:] = 1
        s[ny // 2, :] = 0
    elif name == "seam":
        s[:2, :] = 1
        s[-2:, :] = 1
        s[2:4, :2] = 1          # bumps on both sides of x = 0
        s[2:4, nx - 2:] = 1
        s[ny - 4:ny - 2, 0] = 1
        s[ny - 4:ny - 2, nx - 1] = 1
    return s


@pytest.mark.parametrize("tau", [1.0, 0.8])
@pytest.mark.parametrize("name", ["checkerboard", "isolated nodes", "one-wide channel", "seam"])
def test_degenerate_geometries(lbm, oracle_mod, name, tau):
    """Degenerate geometries against the oracle, both schemes (tau = 1 runs
    the moment step, 0.8 the population step): fields, events and ledgers
    after 1, 5 and 40 steps.  The reaction runs at its limit 4 k_r = 1 (a node
    with four solid axis neighbours consumes all its solute) and the
    threshold is low, so nodes grow within the run."""
    nx, ny = 67, 23
    solid = _degenerate(name, nx, ny)
    rng = np.random.default_rng(nx * ny + len(name))
    fl = solid == 0
    r1 = np.where(fl, 0.8 + 0.2 * rng.random((ny, nx)), 0.0)
    r2 = np.where(fl, 0.05 + 0.1 * rng.random((ny, nx)), 0.0)
    c = np.where(fl, 0.3 + 0.4 * rng.random((ny, nx)), 0.0)
    p = inputs.Params(nx=nx, ny=ny, tau=tau, G=1.6, G_ads1=-0.33, G_ads2=0.33, tau_g=0.65,
                      k_r=0.25, threshold=0.35, accel_x=1e-5)
    PT.say(f"[degenerate] {name} tau {tau}")
    sim = lbm.Sim(p, solid, r1, r2, c, tile=(64, 8))
    orc = oracle_mod.Oracle(p, solid, r1, r2, c)
    for n in (1, 5, 40):
        sim.step(n - orc.steps)
        orc.step(n - orc.steps)
        _fields_cmp(sim, orc, f"{name} tau {tau} step {n}", rho_tol=2e-5, u_tol=2e-5,
                    conc_tol=2e-5, m_tol=1e-6)
        assert PT.event_set(sim.events()) == PT.event_set(orc.events()), (name, n)
    go, oo = sim.observe(), orc.observe()
    for k in ("solute", "precipitate", "solute_removed"):
        assert abs(go[k] - oo[k]) <= 1e-5 * max(1.0, abs(oo[k])), k
    for sc in range(2):
        assert abs(go["mass"][sc] - oo["mass"][sc]) <= 1e-5 * max(1.0, oo["mass"][sc])
        assert abs(go["mass_removed"][sc] - oo["mass_removed"][sc]) <= 1e-5 * max(1.0, oo["mass_removed"][sc])
    assert go["n_solid"] == oo["n_solid"]
    assert len(orc.events()) > 0, name


def test_error_paths(lbm):
    L = lbm
    prob = inputs.config0()
    PT.say("[errors] invalid parameters, workspace, NaN poisoning")
    with pytest.raises(L.LbmError) as e:
        L.Sim(prob.params.replace(tau=0.5), prob.solid, prob.rho1, prob.rho2)
    assert e.value.status == L.LBM_EINVAL
    bad = prob.solid.copy()
    bad[0, 0] = 2
    with pytest.raises(L.LbmError) as e:
        L.Sim(prob.params, bad, prob.rho1, prob.rho2)
    assert e.value.status == L.LBM_EINVAL
    neg = prob.rho1.copy()
    neg[10, 10] = -1.0
    with pytest.raises(L.LbmError):
        L.Sim(prob.params, prob.solid, neg, prob.rho2)
    sim = L.Sim.from_problem(prob)
    with pytest.raises(L.LbmError):
        sim.set_tile(96, 8)
    with pytest.raises(L.LbmError):
        sim.set_load_hint(2)
    with pytest.raises(L.LbmError):
        sim.step(-1)
    # NaN written into the population state -> observe reports and poisons
    sim.step(10)
    blob = sim.save()
    f = np.frombuffer(blob[40:40 + 18 * 256 * 32 * 4], dtype=np.float32).copy().reshape(18, 32, 256)
    f[3, 16, 20] = np.nan
    solid = np.frombuffer(blob[40 + 18 * 256 * 32 * 4:40 + 18 * 256 * 32 * 4 + 256 * 32],
                          dtype=np.uint8).reshape(32, 256)
    sim.load_state(f.astype(np.float64), solid, step=10)
    with pytest.raises(L.LbmError) as e:
        sim.observe()
    assert e.value.status == L.LBM_ENONFINITE
    with pytest.raises(L.LbmError) as e:
        sim.step(1)
    assert e.value.status == L.LBM_ESTATE
    sim.load(blob)          # a good checkpoint clears the poisoned state
    sim.step(5)
    assert sim.observe()["step"] == 15


def test_autotune_cache(lbm, tmp_path, monkeypatch):
    """With LBM_AUTOTUNE_CACHE set, the first autotune times and records its
    choice; a second handle of the same lattice reuses it without timing."""
    path = tmp_path / "tune.jsonl"
    monkeypatch.setenv("LBM_AUTOTUNE_CACHE", str(path))
    prob = inputs.config0()
    PT.say("[autotune cache]")
    a = lbm.Sim.from_problem(prob)
    (tx, sy), ms = a.autotune(steps=2)
    nt = a.load_hint()
    assert nt in (0, 1)
    lines = path.read_text().splitlines()
    assert len(lines) == 1 and f'"tx": {tx}, "sy": {sy}' in lines[0] and f'"nt": {nt}' in lines[0]
    b = lbm.Sim.from_problem(prob)
    b.set_load_hint(1 - nt)
    assert b.autotune(steps=2)[0] == (tx, sy)
    assert len(path.read_text().splitlines()) == 1
    assert b.tile() == (tx, sy) and b.load_hint() == nt


@pytest.mark.parametrize("scheme", ["moments", "populations"])
def test_radii_match_oracle(lbm, oracle_mod, scheme):
    """r_min, r_ave and r_h of Fig. 4 observed on the device equal the
    oracle's (integer counts on identical solid masks) while the walls grow."""
    prob = inputs.capillary_problem(300, 40, 20, seed=5, k_r=0.01, threshold=0.4, D=0.05)
    PT.say(f"[radii] {scheme}: 300x40 reactive capillary, 700 steps")
    sim = lbm.Sim.from_problem(prob, scheme=scheme)
    orc = oracle_mod.Oracle.from_problem(prob)
    go, oo = sim.observe(), orc.observe()
    assert go["r_min"] == go["r_ave"] == go["r_h"] == 20.0
    for n in range(100, 701, 100):
        sim.step(100)
        orc.step(100)
        assert PT.event_set(sim.events()) == PT.event_set(orc.events()), n
        go, oo = sim.observe(), orc.observe()
        for k in ("r_min", "r_ave", "r_h"):
            assert go[k] == oo[k], (n, k, go[k], oo[k])
    assert go["r_h"] <= go["r_ave"] < 20.0 and go["r_min"] < 20.0
