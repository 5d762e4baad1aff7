"""Parameter sweeps over reactive capillaries.

A sweep run advances one capillary for T steps and reports the centreline
front z at the sample times t_j = ceil(j T / nslots), j = 1..nslots, and the
first pore-closure step (Results: front position in the course of time,
Fig. 2; growth of the solid phase and pore closure, Fig. 3).

run_batched advances all runs together (one launch per step, graph replay,
fronts recorded on the device); run_plain does the same runs one after another
with a single-lattice handle each, the way one would without batching.  Both
call only the HIP library.
"""

from __future__ import annotations

import math
import time

import numpy as np

from . import lbm


def sample_times(T: int, nslots: int) -> list:
    return [int(math.ceil(j * T / nslots)) for j in range(1, nslots + 1)]


def run_batched(problems, T: int, nslots: int = 64, *, tile=None, autotune: bool = True,
                device="cuda:0", stream=None, timer=None):
    """Returns (fronts [n, nslots], closure_step [n], seconds, tile)."""
    import torch
    times = sample_times(T, nslots)
    chunk = min(times[0], max(1, times[1] - times[0]))
    b = lbm.Batch(problems, nslots=nslots, device=device, stream=stream)
    if tile is not None:
        b.set_tile(*tile)
    elif autotune:
        b.autotune(steps=3)
    b.set_graph(chunk)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    for j, t in enumerate(times):
        b.step(t - done)
        done = t
        b.record_fronts(j)
    fronts = b.fronts()
    seconds = time.perf_counter() - t0
    closure = np.array([b.observe(i)["closure_step"] for i in range(len(problems))])
    tile = b.tile()
    b.close()
    return fronts, closure, seconds, tile


def run_plain(problems, T: int, nslots: int = 64, *, device="cuda:0"):
    """The same runs one after another, one single-lattice handle per run,
    observing z at every sample time.  Returns (fronts, closure, seconds)."""
    import torch
    times = sample_times(T, nslots)
    fronts = np.zeros((len(problems), nslots))
    closure = np.zeros(len(problems), dtype=np.int64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i, pr in enumerate(problems):
        sim = lbm.Sim.from_problem(pr, device=device)
        done = 0
        for j, t in enumerate(times):
            sim.step(t - done)
            done = t
            fronts[i, j] = sim.observe()["front_z"]
        closure[i] = sim.observe()["closure_step"]
        sim.close()
    seconds = time.perf_counter() - t0
    return fronts, closure, seconds


def targets(problems, fronts, closure, T: int) -> np.ndarray:
    """Per run: z(t_j) / L for the sample times and the closure time / T
    (1.0 when the capillary did not close within T steps)."""
    L = np.array([pr.params.x_out - pr.params.x_in for pr in problems], dtype=np.float64)
    z = fronts / L[:, None]
    c = np.where(closure >= 0, closure / float(T), 1.0)
    return np.concatenate([z, c[:, None]], axis=1)
