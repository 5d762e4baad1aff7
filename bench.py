"""Benchmark of the fused reactive lattice Boltzmann step on one MI355X.

Workload: the 2048x2048 synthetic porous carbon preform (RSA disks of radius
8-24, solid fraction 0.5, wetting reservoir on the left 64 columns, D2Q5
solute with D=0.05, reaction k_r=1e-3, threshold 1, tau=1).  One step = one
full lattice Boltzmann time step (flow + solute + reaction + growth) over all
4,194,304 nodes.  At tau = 1 the library keeps six FP32 moments per node
between steps (the moment scheme); the population scheme (eighteen FP32
populations per node) is timed beside it.  Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
"""

from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published


def wall_adjacent(solid: np.ndarray) -> np.ndarray:
    s = solid != 0
    n = np.zeros(s.shape, dtype=np.int32)
    for ax in (0, 1):
        for sh in (1, -1):
            n += np.roll(s, sh, axis=ax)
    return (~s) & (n > 0)


# Algorithmic HBM bytes per lattice update of the method: 2x9 flow and 5
# solute FP32 populations read and written, 1 mask byte (the FP64 precipitate
# at wall-adjacent nodes adds ~1 B on the preform).  This is the roofline's
# unit for both schemes.
BYTES_PER_LUP_METHOD = 185
# Bytes each scheme itself must move per lattice update.  Population scheme:
# the method's populations.  Moment scheme (tau = 1): 2x3 flow moments
# (rho_s, v_s) and 5 solute populations read and written, 1 mask byte.
BYTES_PER_LUP = {"populations": 185, "moments": 89}
BYTES_PER_WALL_NODE = 16  # FP64 precipitate read and written at wall-adjacent fluid nodes
KERNEL = {"populations": "k_step<true,true,false,double,KIND_POP>",
          "moments": "k_step<true,true,false,double,KIND_MM>"}


def algorithmic_bytes(solid: np.ndarray, scheme: str) -> tuple:
    """Algorithmic HBM bytes of one step: the per-update figure of the scheme
    over all nodes (the unit MLUPS counts) plus 16 B per wall-adjacent fluid
    node.  Also the fluid-only figure (solid nodes touch only their mask
    byte)."""
    b = BYTES_PER_LUP[scheme]
    fluid = int(np.count_nonzero(solid == 0))
    wall = int(np.count_nonzero(wall_adjacent(solid)))
    per_lup = b * solid.size + BYTES_PER_WALL_NODE * wall
    fluid_only = (b - 1) * fluid + solid.size + BYTES_PER_WALL_NODE * wall
    return per_lup, fluid_only, wall


def traffic_key(tile, nt) -> str:
    return f"{tile[0]}x{tile[1]}" + ("/nt" if nt else "")


def measured_traffic(tile, nt, scheme):
    """HBM bytes per launch from the committed PMC summary, only if it was
    taken on this kernel source and scheme, for this launch shape."""
    path = os.path.join(ROOT, "profiles", f"k_step_{scheme}_preform2048_traffic.json")
    src = os.path.join(ROOT, "paper_1309_6726_amd", "csrc", "lbm_kernels.hip")
    try:
        with open(path) as fh:
            rec = json.load(fh)
        with open(src, "rb") as fh:
            sha = hashlib.sha256(fh.read()).hexdigest()
    except OSError:
        return None
    if rec.get("kernel_src_sha256") != sha or rec.get("kernel") != KERNEL[scheme]:
        return None
    t = rec.get("by_tile", {}).get(traffic_key(tile, nt))
    if t is None:
        return None
    return t["fetch_bytes_per_launch"] + t["write_bytes_per_launch"]


def copy_bandwidth(torch, dev, nbytes=1 << 30, reps=10):
    a = torch.empty(nbytes // 4, dtype=torch.float32, device=dev).fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2.0 * nbytes / (ms / 1e3) / 1e9


def cpu_baseline(prob, steps: int, single_steps: int = 5):
    """The oracle on the host: `steps` steps on all OpenMP threads, then
    `single_steps` more on one thread."""
    import ctypes
    from oracle import oracle as O
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    orc = O.Oracle.from_problem(prob)
    orc.step(1)
    t0 = time.perf_counter()
    orc.step(steps)
    dt = time.perf_counter() - t0
    N = prob.params.nx * prob.params.ny
    out = {"value": N * steps / dt / 1e6, "unit": "MLUPS", "cores": threads, "kind": "oracle",
           "sample": f"{steps} steps of the full {prob.params.nx}x{prob.params.ny} preform "
                     f"(after 1 untimed step), FP64, OpenMP {threads} threads, {dt:.1f} s"}
    if single_steps > 0:
        gomp = ctypes.CDLL("libgomp.so.1")
        gomp.omp_set_num_threads(1)
        t0 = time.perf_counter()
        orc.step(single_steps)
        d1 = time.perf_counter() - t0
        gomp.omp_set_num_threads(threads)
        out["single_thread"] = {"value": N * single_steps / d1 / 1e6, "unit": "MLUPS",
                                "steps": single_steps, "seconds": round(d1, 2)}
    return out


def sweep_section(args, torch, dev):
    """Reactive capillary sweep (uneven sizes and parameters): all runs in one
    batch vs the same runs one after another with single-lattice handles."""
    from paper_1309_6726_amd import inputs, sweep
    rows = inputs.sweep_params(0, args.sweep_n)
    probs = [inputs.sweep_problem(r, i, steps=args.sweep_steps) for i, r in enumerate(rows)]
    nodes = sum(int(p.params.nx) * int(p.params.ny) for p in probs)
    T = args.sweep_steps
    info = {}
    fr_b, cl_b, sec_b, tile = sweep.run_batched(probs, T, 64, device=dev, info=info)
    k = min(args.plain_sample, len(probs))
    fr_p, cl_p, sec_p = sweep.run_plain(probs[:k], T, 64, device=dev)
    same = bool(np.array_equal(fr_b[:k], fr_p) and np.array_equal(cl_b[:k], cl_p))
    sample_nodes = sum(int(p.params.nx) * int(p.params.ny) for p in probs[:k])
    # plain time per run, scaled from the sample to the whole sweep by node count
    plain_total = sec_p * nodes / sample_nodes
    return {"runs": len(probs), "steps_per_run": T, "nodes_total": nodes,
            "sampler": "W~U{8..64}, nx~U{256..2048}, ny=W+12, k_r=10^U[-4,-2], "
                       "theta~U[20,40] deg, threshold~U[0.5,2], seed 0",
            "batched": {"seconds": round(sec_b, 3), "setup_s": round(info["setup_s"], 3),
                        "tile": list(tile), "graph_chunk": info["graph_chunk"],
                        "mlups": round(nodes * T / sec_b / 1e6, 1),
                        "runs_per_hour": round(len(probs) / sec_b * 3600, 1)},
            "plain": {"sample_runs": k, "sample_seconds": round(sec_p, 3),
                      "mlups": round(sample_nodes * T / sec_p / 1e6, 1),
                      "runs_per_hour": round(len(probs) / plain_total * 3600, 1)},
            "batched_over_plain": round(plain_total / sec_b, 2),
            "sample_results_identical": same,
            "closed_runs": int(np.count_nonzero(cl_b >= 0))}


def surrogate_section(args, torch, dev, sweep_out):
    """Train the MLP surrogate on batched LB runs (sampler seed 1), score it on
    held-out runs (seed 2) against the LB, and answer queries: network where it
    is in range and confident, LB otherwise (including 32 out-of-range ones).
    The LB answers a query exactly (it is the reference), so the held-out error
    of a query sent to it is 0."""
    from paper_1309_6726_amd import surrogate as S
    T = args.sweep_steps
    rows, x, fr, cl, gen_s = S.generate(1, args.surr_train, T, device=dev)
    rows_t, x_t, fr_t, cl_t, gen_t = S.generate(2, args.surr_test, T, device=dev)
    y = S.make_targets(x, fr, cl, T)
    ens = S.Ensemble(args.surr_members, max_batch=256, max_data=args.surr_train, device=dev)
    t0 = time.perf_counter()
    # the confidence gates are chosen on runs the networks have not seen: the
    # ensemble is trained on all but the last 1/8 of the training runs and its
    # gates are picked on that 1/8; the same ensemble then answers
    nv = len(rows) // 8
    hist = ens.train(x[:-nv], y[:-nv], epochs=args.surr_epochs, lr=2e-3,
                     log_every=args.surr_epochs)
    gates = S.choose_gates(ens, x[-nv:], fr[-nv:], T, target=args.surr_gate_target, p95=0.02)
    train_s = time.perf_counter() - t0
    # raw networks on the held-out runs: one member, and the ensemble mean
    e_one = S.front_error(S.decode(x_t, ens.members[0].predict(x_t).astype(np.float64), T)[0], fr_t)
    f_raw, c_raw = S.decode(x_t, ens.predict(x_t), T)
    e_raw = S.front_error(f_raw, fr_t)
    # gated answers (ensemble where confident, LB elsewhere)
    f_g, c_g, use, net_s, lb_s = S.answer(ens, rows_t, T, gates, device=dev)
    e_g = S.front_error(f_g, fr_t)
    closure_err = np.abs(np.where(c_g >= 0, c_g, T) - np.where(cl_t >= 0, cl_t, T)) / T
    # out-of-range queries must go to the LB
    oor = S.out_of_range_rows(3, 32)
    f_o, c_o, use_o, _, lb_o = S.answer(ens, oor, T, gates, device=dev)
    q = len(rows_t)
    per_query = (net_s + lb_s) / q
    overhead = gen_s + train_s  # LB runs that produce the training data, and training
    batched_rph = sweep_out["batched"]["runs_per_hour"] if sweep_out else None
    plain_rph = sweep_out["plain"]["runs_per_hour"] if sweep_out else None
    rph = 3600.0 / per_query
    rph_charged = q / (net_s + lb_s + overhead) * 3600
    breakeven = None
    if batched_rph:
        gain = 3600.0 / batched_rph - per_query  # seconds saved per query vs batched
        breakeven = int(math.ceil(overhead / gain)) if gain > 0 else None
    return {"train_runs": len(rows), "heldout_runs": q, "steps_per_run": T,
            "data_generation_s": round(gen_s, 2), "heldout_generation_s": round(gen_t, 2),
            "train_s": round(train_s, 2),
            "epochs": args.surr_epochs, "ensemble_members": len(ens.members),
            "final_loss": [h[-1][1] for h in hist],
            "network_only": {"front_err_mean": round(float(e_raw.mean()), 5),
                             "front_err_median": round(float(np.median(e_raw)), 5),
                             "frac_under_2pct": round(float((e_raw < 0.02).mean()), 4),
                             "one_member_err_mean": round(float(e_one.mean()), 5),
                             "one_member_err_median": round(float(np.median(e_one)), 5)},
            "gates": {"min_predicted_travel_lu": gates[0], "max_relative_spread": round(gates[1], 5)},
            "gates_chosen_on": f"{nv} training-seed runs held back from training (answered runs: "
                               f"mean error <= {100 * args.surr_gate_target:g}%, 95th percentile "
                               "<= 2%)",
            "answered_by_network": int(use.sum()),
            "gated": {"frac_under_2pct": round(float((e_g < 0.02).mean()), 4),
                      "front_err_mean": round(float(e_g.mean()), 5),
                      "front_err_p95": round(float(np.quantile(e_g, 0.95)), 5),
                      "front_err_max": round(float(e_g.max()), 5),
                      "network_answers_under_2pct": round(float((e_g[use] < 0.02).mean()), 4)
                      if use.any() else None,
                      "target_met": bool(e_g.mean() < 0.02 and np.quantile(e_g, 0.95) < 0.02),
                      "closure_err_mean": round(float(closure_err.mean()), 5),
                      "network_s": round(net_s, 4), "lb_fallback_s": round(lb_s, 3),
                      "runs_per_hour": round(rph, 1),
                      "runs_per_hour_charging_data_and_training": round(rph_charged, 1),
                      "breakeven_queries_vs_batched": breakeven},
            "out_of_range": {"queries": len(oor), "sent_to_lb": int((~use_o).sum()),
                             "lb_s": round(lb_o, 3)},
            "vs_plain_runs_per_hour": None if not plain_rph else round(rph / plain_rph, 2),
            "vs_batched_runs_per_hour": None if not batched_rph else round(rph / batched_rph, 2)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--start-step", type=int, default=3000,
                    help="steps run (untimed) before autotuning and timing, so the timed "
                         "steps lie where the preform grows (first events near step 770)")
    ap.add_argument("--tile", type=str, default="auto", help="TXxSY or auto")
    ap.add_argument("--load-hint", type=str, default="auto", choices=("auto", "0", "1"),
                    help="with --tile: non-temporal load hint (auto keeps the default, 0)")
    ap.add_argument("--scheme", choices=("auto", "moments", "populations"), default="auto",
                    help="state between steps (auto: moments at tau = 1)")
    ap.add_argument("--compare-steps", type=int, default=1000,
                    help="steps of the other scheme timed for comparison (0: skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=200)
    ap.add_argument("--no-sweep", action="store_true", help="skip the capillary sweep")
    ap.add_argument("--sweep-n", type=int, default=512)
    ap.add_argument("--sweep-steps", type=int, default=10000)
    ap.add_argument("--plain-sample", type=int, default=8)
    ap.add_argument("--no-surrogate", action="store_true", help="skip the surrogate section")
    ap.add_argument("--surr-train", type=int, default=4096)
    ap.add_argument("--surr-test", type=int, default=256)
    ap.add_argument("--surr-epochs", type=int, default=3000)
    ap.add_argument("--surr-members", type=int, default=3, help="networks in the ensemble")
    ap.add_argument("--surr-gate-target", type=float, default=0.01,
                    help="mean front error the gates are chosen for on held-back runs")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run only a 1 GiB device copy and sum (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(use --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1309_6726_amd import inputs, lbm

    dev = torch.device("cuda:0")
    if args.copy_probe:
        # kernels of known traffic for the counter scale: a 1 GiB copy (reads
        # and writes 1 GiB) and a 1 GiB sum (reads 1 GiB, writes 4 bytes)
        a = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        for _ in range(3):
            a.sum()
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_each_way": a.numel() * 4, "launches": 3,
                          "sum_probe_bytes_read": a.numel() * 4}))
        return

    prob = inputs.config2(seed=0)
    p = prob.params
    N = p.nx * p.ny
    scheme = args.scheme
    if scheme == "auto":
        scheme = "moments" if float(p.tau) == 1.0 else "populations"
    stream = torch.cuda.Stream(device=dev)

    def timed_run(scheme, steps, warmup, tile, hint="auto", start=0):
        """Autotune (or set) the launch shape and load hint, advance `start`
        steps in that shape, read the step count and events, then warm up and
        time `steps` steps with HIP events on the library's stream.  The GPU
        runs slower for its first ~100-200 steps after an idle spell of the
        host (clocks ramp up again), so the advance runs right before the
        warm-up and the timed steps, with only a small observe between; the
        host work of the byte count follows the timed steps."""
        sim = lbm.Sim.from_problem(prob, device=dev, stream=stream, scheme=scheme)
        if tile == "auto":
            (tx, sy), _ = sim.autotune(steps=50)
        else:
            tx, sy = (int(v) for v in tile.lower().split("x"))
            sim.set_tile(tx, sy)
            tx, sy = sim.tile()
            if hint != "auto":
                sim.set_load_hint(int(hint))
        nt = sim.load_hint()
        sim.step(start)
        o0 = sim.observe()
        sim.step(warmup)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record(stream)
        sim.step(steps)
        e1.record(stream)
        e1.synchronize()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms = e0.elapsed_time(e1)
        o1 = sim.observe()
        b1 = algorithmic_bytes(sim.fields(("solid",))["solid"].astype(np.uint8), scheme)
        del sim
        return (tx, sy, nt), ms, wall, o0, o1, b1

    with torch.cuda.stream(stream):
        (tx, sy, nt), ms, wall, o0, o1, bytes1 = timed_run(
            scheme, args.steps, args.warmup, args.tile, args.load_hint, args.start_step)
        compare = None
        if args.compare_steps > 0:
            other = "populations" if scheme == "moments" else "moments"
            if other == "populations" or float(p.tau) == 1.0:
                ctile, cms, _, _, _, cb1 = timed_run(other, args.compare_steps, 20, "auto",
                                                     start=args.start_step)
                cstep = cms / args.compare_steps
                cbytes = cb1[0]
                compare = {"scheme": other, "kernel": KERNEL[other], "tile": list(ctile[:2]),
                           "load_hint": ctile[2],
                           "steps": args.compare_steps, "ms_per_step": round(cstep, 5),
                           "mlups": round(N / (cstep / 1e3) / 1e6, 1),
                           "bytes_per_lup": BYTES_PER_LUP[other],
                           "achieved_gbs": round(cbytes / (cstep / 1e3) / 1e9, 1)}
    copy_gbs = copy_bandwidth(torch, dev)
    ms_step = ms / args.steps
    sec_step = ms_step / 1e3
    mlups = N * args.steps / (ms / 1e3) / 1e6
    fluid0 = N - o0["n_solid"]
    method_bytes = BYTES_PER_LUP_METHOD * N
    achieved = method_bytes / sec_step / 1e9
    scheme_bytes = bytes1[0]
    scheme_gbs = scheme_bytes / sec_step / 1e9
    fluid_only = bytes1[1]
    traffic = measured_traffic((tx, sy), nt, scheme)
    cons = abs(o1["solute"] + o1["precipitate"] + o1["solute_removed"] -
               (o0["solute"] + o0["precipitate"] + o0["solute_removed"]))
    out = {
        "metric": "MLUPS & % HBM BW (reactive LB step)",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "porous preform 2048x2048, RSA disks r=8..24, solid fraction "
                               f"{prob.solid_fraction:.3f}, reservoir 64 cols, D2Q5 D=0.05, "
                               "k_r=1e-3, threshold 1, 2-component Shan-Chen D2Q9 tau=1, "
                               f"FP32 state ({scheme}), FP64 arithmetic",
                   "nx": p.nx, "ny": p.ny, "tile": [tx, sy], "load_hint": nt, "scheme": scheme,
                   "timed_from_step": args.start_step + args.warmup,
                   "mflups_fluid": round(fluid0 * args.steps / (ms / 1e3) / 1e6, 1),
                   "wall_adjacent_nodes": bytes1[2],
                   "growth_events_in_warmup_and_timed_steps": int(o1["n_events"] - o0["n_events"]),
                   "solute_ledger_drift": cons, "wall_s": round(wall, 3),
                   "copy_gbs": round(copy_gbs, 1),
                   "frac_of_copy": round(achieved / copy_gbs, 4),
                   "fluid_only_gbs": round(fluid_only / sec_step / 1e9, 1)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None if traffic is None else int(traffic),
                     "kernel": KERNEL[scheme],
                     "bytes_per_lup": BYTES_PER_LUP_METHOD,
                     "algorithmic_bytes_per_launch": int(method_bytes),
                     "avg_launch_ms": round(ms_step, 5),
                     "basis": "the method's 185 B per lattice update (populations) x all "
                              "nodes; the moment scheme moves fewer bytes for the same update",
                     "scheme_bytes": {"bytes_per_lup": BYTES_PER_LUP[scheme],
                                      "bytes_per_wall_node": BYTES_PER_WALL_NODE,
                                      "bytes_per_launch": int(scheme_bytes),
                                      "achieved": round(scheme_gbs, 1),
                                      "frac": round(scheme_gbs / HBM_PEAK_GBS, 4)},
                     "counter_gbs": None if traffic is None else round(traffic / sec_step / 1e9, 1)},
    }
    if compare is not None:
        out["other_scheme"] = compare
    if not args.no_sweep:
        out["sweep"] = sweep_section(args, torch, dev)
    if not args.no_surrogate:
        out["surrogate"] = surrogate_section(args, torch, dev, out.get("sweep"))
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
