"""Helpers for GPU-vs-oracle parity tests (test infrastructure).

The GPU stores the state in FP32 and computes in FP64; the oracle is FP64
throughout.  Tolerances:
  * densities: max |rho_gpu - rho_cpu| <= 1e-5 (relative to the majority
    density 1) after 1000-2000 steps;
  * barycentric velocity: <= 1e-6 absolute;
  * total mass drift: relative 1e-6 (sums are taken in FP64 on both sides);
  * front position: 0.01 lattice units;
  * growth events: identical sets of (x, y, step).  The contract configs
    (the 256x32 and 1024x64 capillaries, the 2048x2048 preform) allow no
    exception.  Long reactive runs beyond them may opt into certified ties:
    a disagreement passes only if the oracle's margin |m - threshold| at that
    step is within 10x the largest precipitate difference at the previous
    window boundary (floor 1e-9), i.e. the two precisions straddle the
    threshold; the oracle then adopts the GPU's decision and both continue.
"""

from __future__ import annotations

import sys

import numpy as np

RHO_TOL = 1e-5
U_TOL = 1e-6
MASS_TOL = 1e-6
Z_TOL = 0.01


def say(*args):
    print(*args, flush=True)
    sys.stdout.flush()


def compare_fields(gf: dict, of: dict, *, rho_tol=RHO_TOL, u_tol=U_TOL, conc_tol=1e-5,
                   m_tol=1e-5, where=""):
    solid_g = gf["solid"] != 0
    solid_o = of["solid"] != 0
    assert np.array_equal(solid_g, solid_o), f"{where}: solid masks differ"
    fl = ~solid_o
    out = {}
    for k in ("rho1", "rho2"):
        d = np.abs(gf[k] - of[k])[fl].max(initial=0.0)
        out[k] = d
        assert d <= rho_tol, f"{where}: {k} differs by {d:.3e}"
    for k in ("ux", "uy"):
        d = np.abs(gf[k] - of[k])[fl].max(initial=0.0)
        out[k] = d
        assert d <= u_tol, f"{where}: {k} differs by {d:.3e}"
    if "conc" in gf:
        d = np.abs(gf["conc"] - of["conc"])[fl].max(initial=0.0)
        out["conc"] = d
        assert d <= conc_tol, f"{where}: conc differs by {d:.3e}"
    if "precip" in gf:
        d = np.abs(gf["precip"] - of["m"]).max(initial=0.0)
        out["m"] = d
        assert d <= m_tol, f"{where}: precipitate differs by {d:.3e}"
    return out


def gpu_fields(sim) -> dict:
    return sim.fields()


def event_set(ev) -> set:
    return {(int(e["x"]), int(e["y"]), int(e["step"])) for e in ev}


def run_windows(sim, orc, nsteps: int, window: int, *, threshold=None, allow_ties=False,
                field_check=None, log=say):
    """Advance GPU and oracle in lock-step windows and compare the growth-event
    sets at every window boundary.  Without allow_ties any difference fails,
    naming the first events that differ; with it, each difference must be a
    certified tie (module docstring), which the oracle then adopts.  Returns
    (n_events, n_ties, max precipitate difference at the last boundary,
    oracle)."""
    eps = 1e-9
    ties = 0
    done = 0
    max_dm = 0.0
    gset = set()
    while done < nsteps:
        n = min(window, nsteps - done)
        start = orc.clone() if allow_ties else None
        sim.step(n)
        orc.step(n)
        gset = event_set(sim.events())
        oset = event_set(orc.events())
        rounds = 0
        while gset != oset:
            diff = sorted(gset ^ oset, key=lambda e: (e[2], e[1], e[0]))
            if not allow_ties:
                om = orc.fields()["m"]
                detail = ", ".join(f"({x},{y}) step {s} {'GPU' if (x, y, s) in gset else 'oracle'} "
                                   f"only, oracle m now {om[y, x]:.9f}" for (x, y, s) in diff[:5])
                raise AssertionError(f"growth events differ in the window ending at step "
                                     f"{done + n}: {len(gset - oset)} GPU-only, "
                                     f"{len(oset - gset)} oracle-only; {detail}")
            # the earliest disagreements decide; later ones may be their
            # consequences, so the window is re-run after adopting them
            rounds += 1
            assert rounds <= 20, "too many rounds of certified ties in one window"
            first = [e for e in diff if e[2] == diff[0][2]]
            for (x, y, s) in first:
                probe = start.clone()
                probe.step(s - probe.steps)
                margin = abs(probe.fields()["m"][y, x] - threshold)
                tol = max(eps, 10.0 * max_dm)
                assert margin <= tol, (f"uncertified event mismatch at ({x},{y}) step {s}: "
                                       f"oracle margin {margin:.3e} > {tol:.3e}")
                log(f"  certified tie at ({x},{y}) step {s}: oracle margin {margin:.2e} <= {tol:.2e}")
                start.override(x, y, s, (x, y, s) in gset)
            ties += len(first)
            orc = start.clone()
            orc.step(n)
            oset = event_set(orc.events())
        gm = sim.fields(("precip", "solid"))["precip"]
        om = orc.fields()["m"]
        max_dm = float(np.abs(gm - om).max())
        if field_check is not None:
            field_check(done + n, sim, orc)
        done += n
        log(f"  step {done}: {len(gset)} events, max |dm| {max_dm:.2e}, ties {ties}")
    return len(gset), ties, max_dm, orc
