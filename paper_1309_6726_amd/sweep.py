"""Parameter sweeps over reactive capillaries.

A sweep run advances one capillary for T steps and reports the centreline
front z at the sample times t_j = ceil(j T / nslots), j = 1..nslots, and the
first pore-closure step (Results: front position in the course of time,
Fig. 2; growth of the solid phase and pore closure, Fig. 3).

run_batched advances all runs together (one launch per step, graph replay,
fronts recorded on the device); run_plain does the same runs one after another
with a single-lattice handle each, the way one would without batching.  Both
call only the HIP library, and both are timed from before their handles are
built to the results on the host.
"""

from __future__ import annotations

import math
import time

import numpy as np

from . import lbm


def sample_times(T: int, nslots: int) -> list:
    return [int(math.ceil(j * T / nslots)) for j in range(1, nslots + 1)]


def run_batched(problems, T: int, nslots: int = 64, *, tile=None, autotune: bool = True,
                device="cuda:0", stream=None, info=None):
    """Returns (fronts [n, nslots], closure_step [n], seconds, tile).

    `seconds` runs from before the batch is built (host inputs copied in,
    initial state, launch-shape search, graph capture) to the fronts back on
    the host, as run_plain times its per-run handles; with a dict `info` the
    set-up part is also reported there as info["setup_s"]."""
    import torch
    times = sample_times(T, nslots)
    chunk = min(times[0], max(1, times[1] - times[0]))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b = lbm.Batch(problems, nslots=nslots, device=device, stream=stream)
    if tile is not None:
        b.set_tile(*tile)
    elif autotune:
        b.autotune(steps=3)
    b.set_graph(chunk)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    done = 0
    for j, t in enumerate(times):
        b.step(t - done)
        done = t
        b.record_fronts(j)
    fronts = b.fronts()
    seconds = time.perf_counter() - t0
    if info is not None:
        info["setup_s"] = t1 - t0
        info["graph_chunk"] = chunk
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


def main(argv=None):
    """Run a batched sweep of the capillary sampler's runs and print one JSON
    line (seconds, aggregate MLUPS, runs/hour); with --plain K also the first
    K runs one after another.

      python -m paper_1309_6726_amd.sweep [--runs N] [--steps T] [--seed S]
    """
    import argparse
    import json

    from . import inputs
    ap = argparse.ArgumentParser(prog="python -m paper_1309_6726_amd.sweep")
    ap.add_argument("--runs", type=int, default=512)
    ap.add_argument("--steps", type=int, default=10_000)
    ap.add_argument("--seed", type=int, default=0, help="sampler seed")
    ap.add_argument("--nslots", type=int, default=64, help="front samples per run")
    ap.add_argument("--tile", type=str, default="auto", help="TXxSY or auto")
    ap.add_argument("--plain", type=int, default=0, help="also run the first K runs one by one")
    args = ap.parse_args(argv)
    rows = inputs.sweep_params(args.seed, args.runs)
    probs = [inputs.sweep_problem(r, i, steps=args.steps) for i, r in enumerate(rows)]
    nodes = sum(int(p.params.nx) * int(p.params.ny) for p in probs)
    tile = None if args.tile == "auto" else tuple(int(v) for v in args.tile.lower().split("x"))
    fr, cl, sec, tile = run_batched(probs, args.steps, args.nslots, tile=tile)
    out = {"runs": len(probs), "steps": args.steps, "seed": args.seed, "nodes": nodes,
           "tile": list(tile), "seconds": round(sec, 4),
           "ms_per_step": round(1e3 * sec / args.steps, 5),
           "mlups": round(nodes * args.steps / sec / 1e6, 1),
           "runs_per_hour": round(len(probs) / sec * 3600, 1),
           "closed_runs": int((cl >= 0).sum())}
    if args.plain > 0:
        k = min(args.plain, len(probs))
        frp, clp, secp = run_plain(probs[:k], args.steps, args.nslots)
        out["plain"] = {"runs": k, "seconds": round(secp, 4),
                        "identical": bool(np.array_equal(fr[:k], frp) and np.array_equal(cl[:k], clp))}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
