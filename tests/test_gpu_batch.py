"""Batched sweeps through the C ABI: every instance of a batch must compute
exactly what a single-lattice run computes for it (bit for bit), in direct and
graph-replay mode, and match the FP64 oracle."""

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


def _problems(n=5, seed=11):
    """Uneven reactive capillaries from the sweep sampler, shortened and made
    fast-reacting so growth events happen within a few hundred steps."""
    rows = inputs.sweep_params(seed, n)
    probs = []
    for i, r in enumerate(rows):
        W, nx, k, th, thr = r
        r = (W, 256 + (int(nx) % 300), 0.005 + 0.01 * (i % 3), th, 0.3 + 0.1 * (i % 4))
        probs.append(inputs.sweep_problem(r, instance=i))
    return probs


def _same_fields(a, b, where):
    for k in a:
        assert np.array_equal(a[k], b[k]), f"{where}: field {k} differs"


def test_batch_equals_single_runs_bitwise(lbm):
    probs = _problems()
    PT.say(f"[batch] {len(probs)} instances, sizes {[p.solid.shape for p in probs]}: 600 steps")
    batch = lbm.Batch(probs, tile=(128, 24))
    batch.step(600)
    total_events = 0
    for i, pr in enumerate(probs):
        sim = lbm.Sim.from_problem(pr)
        sim.step(600)
        _same_fields(batch.fields(i), sim.fields(), f"instance {i}")
        assert PT.event_set(batch.events(i)) == PT.event_set(sim.events())
        assert batch.observe(i) == sim.observe()
        total_events += len(sim.events())
    assert total_events > 0


def test_batch_graph_replays_match_direct(lbm):
    """Graph of 100 captured steps replayed 5 times, with observes and field
    copies between the replays; every replay equals direct launches."""
    probs = _problems(4, seed=12)
    PT.say("[batch graph] chunk 100 x 5 replays vs direct launches")
    g = lbm.Batch(probs, tile=(64, 16), graph_chunk=100)
    d = lbm.Batch(probs, tile=(64, 16))
    for rep in range(5):
        g.step(100)
        d.step(100)
        for i in range(len(probs)):
            assert g.observe(i) == d.observe(i), (rep, i)
            _same_fields(g.fields(i), d.fields(i), f"replay {rep} instance {i}")
    g.step(137)   # one replay plus 37 direct steps
    d.step(137)
    for i in range(len(probs)):
        _same_fields(g.fields(i), d.fields(i), f"tail instance {i}")
        assert PT.event_set(g.events(i)) == PT.event_set(d.events(i))


def test_batch_front_table(lbm):
    probs = _problems(6, seed=13)
    PT.say("[batch fronts] 4 slots")
    b = lbm.Batch(probs, nslots=4, graph_chunk=50)
    expect = np.zeros((len(probs), 4))
    for s in range(4):
        b.step(150)
        b.record_fronts(s)
        for i in range(len(probs)):
            expect[i, s] = b.observe(i)["front_z"]
    tab = b.fronts()
    assert np.array_equal(tab, expect)
    assert np.all(tab[:, -1] >= 0.0)


def test_batch_instance_matches_oracle(lbm, oracle_mod):
    probs = _problems(3, seed=14)
    PT.say("[batch vs oracle] 500 steps")
    b = lbm.Batch(probs)
    b.step(500)
    for i, pr in enumerate(probs):
        orc = oracle_mod.Oracle.from_problem(pr)
        orc.step(500)
        PT.compare_fields(b.fields(i), orc.fields(), where=f"batch instance {i}")
        assert PT.event_set(b.events(i)) == PT.event_set(orc.events())
        assert abs(b.observe(i)["front_z"] - orc.observe()["front_z"]) <= PT.Z_TOL


def test_batch_autotune_resets_state(lbm):
    probs = _problems(3, seed=15)
    PT.say("[batch autotune]")
    a = lbm.Batch(probs)
    (tx, sy), ms = a.autotune(steps=3)
    assert tx in (64, 128, 256) and sy >= 8 and ms > 0
    a.step(200)
    ref = lbm.Batch(probs, tile=(64, 8))
    ref.step(200)
    for i in range(len(probs)):
        _same_fields(a.fields(i), ref.fields(i), f"instance {i}")


def test_batch_rejects_mixed_switches(lbm):
    probs = _problems(2, seed=16)
    probs[1].params = probs[1].params.replace(G=1.5)
    with pytest.raises(lbm.LbmError) as e:
        lbm.Batch(probs)
    assert e.value.status == lbm.LBM_EINVAL


@pytest.mark.timeout(900)
def test_sweep_rows_graph_replay_match_oracle(lbm, oracle_mod):
    """Six runs of the benchmark's sweep (sampler seed 0, parameters as drawn:
    the narrowest and widest channel, the slowest and fastest reaction, the
    longest capillary and one more) batched as the sweep runs them (graph
    replay, fronts recorded on the device at 16 sample times of 2000 steps)
    against the oracle: every recorded front within 0.01 lu, growth events and
    closure steps exact; fields within the parity tolerances at step 1000 (the
    step the contract fixes them at) and within the random-state bounds (2e-5)
    at step 2000, where the run with the fastest reaction in a narrow channel
    reaches 1.1e-5 in the density."""
    from paper_1309_6726_amd import sweep
    rows = inputs.sweep_params(0, 512)
    pick = [int(np.argmin(rows[:, 0])), int(np.argmax(rows[:, 0])), int(np.argmin(rows[:, 2])),
            int(np.argmax(rows[:, 2])), int(np.argmax(rows[:, 1])), 7]
    probs = [inputs.sweep_problem(rows[i], i) for i in pick]
    T, NS = 2000, 16
    times = sweep.sample_times(T, NS)
    PT.say(f"[sweep rows vs oracle] instances {pick}, sizes {[p.solid.shape for p in probs]}, "
           f"{T} steps, graph chunk {times[0]}")
    b = lbm.Batch(probs, nslots=NS, graph_chunk=times[0])
    orcs = [oracle_mod.Oracle.from_problem(p) for p in probs]
    oz = np.zeros((len(probs), NS))
    done = 0
    for j, t in enumerate(times):
        b.step(t - done)
        b.record_fronts(j)
        for i, o in enumerate(orcs):
            o.step(t - done)
            oz[i, j] = o.observe()["front_z"]
            if t == 1000:
                PT.compare_fields(b.fields(i), o.fields(), where=f"sweep run {pick[i]} step 1000")
        done = t
    gz = b.fronts()
    assert np.abs(gz - oz).max() <= PT.Z_TOL, float(np.abs(gz - oz).max())
    nev = 0
    for i, o in enumerate(orcs):
        ge, oe = PT.event_set(b.events(i)), PT.event_set(o.events())
        assert ge == oe, (pick[i], len(ge - oe), len(oe - ge))
        nev += len(ge)
        assert b.observe(i)["closure_step"] == o.observe()["closure_step"]
        PT.compare_fields(b.fields(i), o.fields(), rho_tol=2e-5, u_tol=2e-5, conc_tol=2e-5,
                          where=f"sweep run {pick[i]} step 2000")
    PT.say(f"  fronts within {np.abs(gz - oz).max():.2e} lu, {nev} growth events identical")
    assert nev > 0
    b.close()
