"""Seeded synthetic inputs: geometry, initial densities and run parameters.

This module is the one piece shared by the HIP path and the FP64 oracle.  It
builds host arrays (solid mask, the two initial component densities, the
initial solute concentration) and plain parameter records; it holds none of
the lattice Boltzmann arithmetic.  Both sides turn these arrays into
populations themselves.

Sources for the set-up (Sergi, Grossi, Leidi, Ortona, "Lattice Boltzmann
simulation of the surface growth effects for the infiltration of molten Si in
carbon preforms"):
  * a single 2D capillary of height H and length L, wetting Si on one side
    ("red" component) and the other substance ("blue") on the other
    (Fig. 1 caption; Results, text around Eq. (1));
  * the two fluids have almost the same density (Introduction);
  * the target contact angle is 30 degrees (Introduction);
  * reaction-rate constant k_r in lu/ts is the only reactivity knob and mass
    precipitates on the surface until a threshold turns the node solid
    (section "LB models").
Array convention: 2D arrays of shape (ny, nx), node index y*nx + x.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(state: np.ndarray) -> np.ndarray:
    """SplitMix64 output for each 64-bit state (Steele, Lea & Flood 2014).

    One call advances the state by the golden gamma and returns the mixed
    value; here the state is a counter so every draw is independent of the
    order in which draws are made."""
    with np.errstate(over="ignore"):
        z = np.asarray(state, dtype=np.uint64) + GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def uniform53(seed: int, counters: np.ndarray) -> np.ndarray:
    """Uniform doubles in [0, 1) with 53 random bits, one per counter.

    draw(c) = (SplitMix64(seed XOR c*gamma) >> 11) * 2^-53."""
    with np.errstate(over="ignore"):
        c = np.asarray(counters, dtype=np.uint64)
        z = splitmix64(np.uint64(seed) ^ (c * GOLDEN))
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


# --------------------------------------------------------------------------
# Model constants.  G and the adhesion strength are calibrated on the FP64
# oracle (the coexisting density pair and the 30 degree contact angle); the
# calibration script lives with the test fixtures and the tests re-check it.
# --------------------------------------------------------------------------
RHO_HI = 1.0        # majority density of a component inside its own phase
RHO_LO = 0.05       # minority density (the two phases have nearly equal total density)
NOISE = 1.0e-3      # amplitude of the additive uniform noise on each density
G_COH = 1.6         # fluid-fluid cohesion strength between unlike components
G_ADS_30 = 0.3314   # |adhesion| giving 30 degrees; wetting component gets -G_ADS
TAU = 1.0           # flow BGK relaxation time (both components)
D_SOLUTE = 0.05     # solute diffusivity -> tau_g = 1/2 + 3 D on D2Q5
C0 = 1.0            # initial solute concentration in the wetting phase


# Static contact angle (degrees) against |adhesion| at G_COH, tau = 1: a
# wetting slug in a 20-wide channel, circle fit of the phi = 1/2 contour.
ANGLE_TABLE = (
    (0.28, 41.12),
    (0.29, 39.01),
    (0.30, 36.94),
    (0.31, 34.88),
    (0.32, 32.74),
    (0.33, 30.39),
    (0.34, 27.60),
    (0.35, 23.91),
    (0.36, 19.28),
    (0.37, 13.94),
)


def adhesion_for_angle(theta_deg: float) -> float:
    """|G_ads| that gives the static contact angle theta (linear interpolation
    in ANGLE_TABLE; valid for 14 to 41 degrees)."""
    ga = np.array([a for a, _ in ANGLE_TABLE])
    th = np.array([t for _, t in ANGLE_TABLE])
    if not (th.min() <= theta_deg <= th.max()):
        raise ValueError("contact angle outside the calibrated range")
    return float(np.interp(theta_deg, th[::-1], ga[::-1]))


def tau_g_for(D: float) -> float:
    return 0.5 + 3.0 * D


@dataclasses.dataclass
class Params:
    """Run parameters, mirroring the C struct accepted by both sides."""
    nx: int
    ny: int
    tau: float = TAU
    G: float = G_COH
    G_ads1: float = -G_ADS_30
    G_ads2: float = +G_ADS_30
    tau_g: float = 0.0          # 0 disables the solute lattice
    k_r: float = 0.0            # 0 disables the surface reaction and growth
    threshold: float = 1.0      # precipitated mass that turns a node solid (strict >)
    accel_x: float = 0.0        # uniform body acceleration (tests only)
    accel_y: float = 0.0
    x_in: int = 0               # capillary descriptor for the front / growth observables
    x_out: int = 0
    y0: int = 0
    W: int = 0                  # 0: no capillary observables
    c_eq: float = 0.0           # saturation concentration of the reaction (0: plain first order)
    c_hold: float = 0.0         # held solute concentration of the source region
    hold_x: int = 0             # source region x < hold_x (0: no source)
    solute_q: int = 0           # solute lattice: 0/5 D2Q5, 4 D2Q4

    def replace(self, **kw) -> "Params":
        return dataclasses.replace(self, **kw)


@dataclasses.dataclass
class Problem:
    """A complete input: parameters plus host arrays (shape (ny, nx))."""
    params: Params
    solid: np.ndarray           # uint8 0/1
    rho1: np.ndarray            # float64, 0 at solid nodes
    rho2: np.ndarray
    conc: np.ndarray | None     # float64 or None when the solute lattice is off
    name: str = ""
    steps: int = 0


# --------------------------------------------------------------------------
# Geometry
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Capillary:
    solid: np.ndarray
    wet: np.ndarray             # bool: initially in the wetting phase
    x_in: int
    x_out: int
    y0: int
    W: int

    @property
    def L(self) -> int:
        return self.x_out - self.x_in


def capillary(nx: int, ny: int, W: int, x_in: int | None = None,
              x_out: int | None = None) -> Capillary:
    """Straight capillary between solid blocks, periodic domain.

    Channel rows y0..y0+W-1 with y0 = (ny-W)//2.  In the capillary section
    x_in <= x < x_out every other row is solid (rows y0-1 and y0+W are the
    wall faces).  Left of x_in lies the wetting reservoir, right of x_out the
    non-wetting one; they meet across the periodic seam at a flat interface."""
    if W < 1 or W > ny - 2:
        raise ValueError("channel width must leave at least one solid row")
    x_in = nx // 3 if x_in is None else x_in
    x_out = nx - 32 if x_out is None else x_out
    if not (0 < x_in < x_out <= nx):
        raise ValueError("bad capillary section")
    y0 = (ny - W) // 2
    solid = np.zeros((ny, nx), dtype=np.uint8)
    rows = np.ones(ny, dtype=bool)
    rows[y0:y0 + W] = False
    solid[np.ix_(rows, np.arange(x_in, x_out))] = 1
    wet = np.zeros((ny, nx), dtype=bool)
    wet[:, :x_in] = True
    wet &= solid == 0
    return Capillary(solid, wet, x_in, x_out, y0, W)


def preform_rsa(nx: int = 2048, ny: int = 2048, seed: int = 0,
                x_lo: int = 64, x_hi: int = 1984, r_min: float = 8.0,
                r_max: float = 24.0, target: float = 0.5, gap: float = 2.0,
                max_attempts: int = 10_000_000, batch: int = 0):
    """Porous preform by random sequential addition of non-overlapping disks.

    Radii U[r_min, r_max]; centres x in [x_lo + r, x_hi - r), y in [0, ny)
    periodic in y.  A candidate is accepted if its distance to every placed
    disk is at least r_i + r_j + gap.  Node (x, y) is solid when it lies in a
    disk ((x-cx)^2 + dy^2 <= r^2, dy periodic).  Stops when the solid node
    fraction of the preform region reaches `target`; raises if that takes
    more than `max_attempts` candidates.  Candidate k draws (r, cx, cy) from
    counters 3k, 3k+1, 3k+2 of the seeded SplitMix64 stream, and candidates
    are tested strictly in k order, so the result does not depend on `batch`
    (0 = adapt the batch to the acceptance rate).

    Returns (solid uint8 (ny, nx), solid_fraction, n_disks, attempts)."""
    region = (x_hi - x_lo) * ny
    solid = np.zeros((ny, nx), dtype=np.uint8)
    # cell grid for the overlap test: any conflicting pair of centres lies
    # in the same or an adjacent cell (cell edge >= 2 r_max + gap)
    cs = 2.0 * r_max + gap
    ncx = int(math.ceil(nx / cs))
    ncy = max(1, int(ny // cs))
    chy = ny / ncy
    K = 24
    gx = np.full((ncx, ncy, K), 1.0e9)
    gy = np.zeros((ncx, ncy, K))
    gr = np.zeros((ncx, ncy, K))
    gn = np.zeros((ncx, ncy), dtype=np.int64)
    offs = [(a, b) for a in (-1, 0, 1) for b in (-1, 0, 1)]
    n_solid = 0
    n_disks = 0
    attempts = 0
    adapt = batch <= 0
    batch = 64 if adapt else batch
    while n_solid < target * region:
        if attempts >= max_attempts:
            raise RuntimeError(f"RSA did not reach solid fraction {target} "
                               f"in {max_attempts} attempts")
        k = np.arange(attempts, attempts + batch, dtype=np.uint64)
        u = uniform53(seed, np.stack([3 * k, 3 * k + 1, 3 * k + 2]))
        r = r_min + (r_max - r_min) * u[0]
        x = (x_lo + r) + u[1] * (x_hi - x_lo - 2 * r)
        y = u[2] * ny
        icx = np.minimum((x / cs).astype(np.int64), ncx - 1)
        icy = np.minimum((y / chy).astype(np.int64), ncy - 1)
        ok = np.ones(batch, dtype=bool)
        for (a, b) in offs:
            cxs = icx + a
            valid = (cxs >= 0) & (cxs < ncx)
            cxs = np.clip(cxs, 0, ncx - 1)
            cys = np.mod(icy + b, ncy)
            px = np.where(valid[:, None], gx[cxs, cys], 1.0e9)
            dy = np.abs(y[:, None] - gy[cxs, cys])
            dy = np.minimum(dy, ny - dy)
            need = r[:, None] + gr[cxs, cys] + gap
            ok &= ~np.any((x[:, None] - px) ** 2 + dy * dy < need * need, axis=1)
        done = False
        placed = []
        for i in np.nonzero(ok)[0]:
            good = True
            for (px, py, pr) in placed:
                ddy = abs(y[i] - py)
                ddy = min(ddy, ny - ddy)
                if (x[i] - px) ** 2 + ddy ** 2 < (r[i] + pr + gap) ** 2:
                    good = False
                    break
            if not good:
                continue
            placed.append((x[i], y[i], r[i]))
            c1, c2 = icx[i], icy[i]
            if gn[c1, c2] >= K:
                raise RuntimeError("RSA cell overflow")
            gx[c1, c2, gn[c1, c2]] = x[i]
            gy[c1, c2, gn[c1, c2]] = y[i]
            gr[c1, c2, gn[c1, c2]] = r[i]
            gn[c1, c2] += 1
            n_disks += 1
            n_solid += _raster_disk(solid, x[i], y[i], r[i])
            if n_solid >= target * region:
                attempts += int(i) + 1
                done = True
                break
        if not done:
            attempts += batch
        if adapt:   # aim for a few tens of acceptances per batch
            batch = int(min(16384, max(64, 32 * batch / max(1, len(placed)))))
    return solid, n_solid / region, n_disks, attempts


def _raster_disk(solid: np.ndarray, cx: float, cy: float, r: float) -> int:
    ny, nx = solid.shape
    x0 = int(math.ceil(cx - r)); x1 = int(math.floor(cx + r))
    y0 = int(math.ceil(cy - r)); y1 = int(math.floor(cy + r))
    xs = np.arange(x0, x1 + 1)
    ys = np.arange(y0, y1 + 1)
    inside = (xs[None, :] - cx) ** 2 + (ys[:, None] - cy) ** 2 <= r * r
    yy = np.mod(ys, ny)
    sub = solid[np.ix_(yy, xs)]
    added = int(np.count_nonzero(inside & (sub == 0)))
    sub[inside] = 1
    solid[np.ix_(yy, xs)] = sub
    return added


# --------------------------------------------------------------------------
# Initial fields
# --------------------------------------------------------------------------
def init_fields(solid: np.ndarray, wet: np.ndarray, seed: int,
                rho_hi: float = RHO_HI, rho_lo: float = RHO_LO,
                noise: float = NOISE, c0: float | None = C0):
    """Initial densities (rho1 wetting, rho2 other) and solute concentration.

    Fluid nodes of the wetting region get (rho_hi, rho_lo), the rest
    (rho_lo, rho_hi); each component at each fluid node gets additive noise
    noise*(2U-1) with U drawn from counter 2*idx + sigma - 1 (sigma = 1, 2).
    Solute: c0 on fluid wetting nodes, 0 elsewhere (None if c0 is None)."""
    ny, nx = solid.shape
    fluid = solid == 0
    idx = np.arange(nx * ny, dtype=np.uint64).reshape(ny, nx)
    u1 = uniform53(seed, 2 * idx)
    u2 = uniform53(seed, 2 * idx + np.uint64(1))
    rho1 = np.where(wet, rho_hi, rho_lo) + noise * (2.0 * u1 - 1.0)
    rho2 = np.where(wet, rho_lo, rho_hi) + noise * (2.0 * u2 - 1.0)
    rho1 = np.where(fluid, rho1, 0.0)
    rho2 = np.where(fluid, rho2, 0.0)
    conc = None
    if c0 is not None:
        conc = np.where(fluid & wet, c0, 0.0).astype(np.float64)
    return rho1, rho2, conc


# --------------------------------------------------------------------------
# The workloads
# --------------------------------------------------------------------------
def capillary_problem(nx: int, ny: int, W: int, seed: int = 0, *,
                      k_r: float = 0.0, threshold: float = 1.0,
                      D: float | None = None, G_ads: float = G_ADS_30,
                      steps: int = 0, name: str = "",
                      x_in: int | None = None, x_out: int | None = None,
                      noise: float = NOISE) -> Problem:
    cap = capillary(nx, ny, W, x_in, x_out)
    solute = D is not None
    rho1, rho2, conc = init_fields(cap.solid, cap.wet, seed, noise=noise,
                                   c0=C0 if solute else None)
    p = Params(nx=nx, ny=ny, G_ads1=-G_ads, G_ads2=+G_ads,
               tau_g=tau_g_for(D) if solute else 0.0, k_r=k_r,
               threshold=threshold, x_in=cap.x_in, x_out=cap.x_out,
               y0=cap.y0, W=W)
    return Problem(p, cap.solid, rho1, rho2, conc, name=name, steps=steps)


def config0(seed: int = 0) -> Problem:
    """256x32 capillary, W=20, no reaction, no solute, 2000 steps."""
    return capillary_problem(256, 32, 20, seed, steps=2000,
                             name="capillary 256x32 W=20, no reaction")


def config1(seed: int = 0) -> Problem:
    """1024x64 reactive capillary, W=48, D=0.05, k_r=1e-3, threshold 1, 50k steps."""
    return capillary_problem(1024, 64, 48, seed, k_r=1e-3, threshold=1.0,
                             D=D_SOLUTE, steps=50_000,
                             name="reactive capillary 1024x64 W=48")


_PREFORM_CACHE: dict = {}


def preform_problem(nx: int = 2048, ny: int = 2048, seed: int = 0, *,
                    reservoir: int = 64, buffer: int = 64, k_r: float = 1e-3,
                    threshold: float = 1.0, D: float = D_SOLUTE,
                    steps: int = 20_000, gap: float = 2.0) -> Problem:
    """Porous carbon preform: wetting reservoir x < reservoir, non-wetting
    buffer x >= nx - buffer, RSA disks in between (solid fraction 0.5)."""
    key = (nx, ny, seed, reservoir, buffer, gap)
    if key not in _PREFORM_CACHE:
        solid, frac, nd, att = preform_rsa(nx, ny, seed, x_lo=reservoir,
                                           x_hi=nx - buffer, gap=gap)
        _PREFORM_CACHE[key] = (solid, frac, nd, att)
    solid, frac, nd, att = _PREFORM_CACHE[key]
    wet = np.zeros((ny, nx), dtype=bool)
    wet[:, :reservoir] = True
    rho1, rho2, conc = init_fields(solid, wet, seed, c0=C0)
    p = Params(nx=nx, ny=ny, tau_g=tau_g_for(D), k_r=k_r, threshold=threshold)
    prob = Problem(p, solid.copy(), rho1, rho2, conc, steps=steps,
                   name=f"porous preform {nx}x{ny} RSA disks r=8..24, "
                        f"solid fraction {frac:.3f}")
    prob.solid_fraction = frac  # type: ignore[attr-defined]
    prob.n_disks = nd           # type: ignore[attr-defined]
    return prob


def config2(seed: int = 0) -> Problem:
    return preform_problem(seed=seed)


# --------------------------------------------------------------------------
# Parameter sweeps over uneven capillaries
# --------------------------------------------------------------------------
SWEEP_RANGES = {"W": (8, 64), "nx": (256, 2048), "log10_k": (-4.0, -2.0),
                "theta": (20.0, 40.0), "threshold": (0.5, 2.0)}


def sweep_params(seed: int, n: int) -> np.ndarray:
    """n parameter rows (W, nx, k_r, theta_deg, threshold) for the capillary
    sweep: W ~ U{8..64}, nx ~ U{256..2048}, k_r = 10^U[-4,-2],
    theta ~ U[20, 40] degrees, threshold ~ U[0.5, 2.0].  Row i draws counters
    5i..5i+4 of the seeded SplitMix64 stream."""
    i = np.arange(n, dtype=np.uint64)
    u = uniform53(seed, np.stack([5 * i + np.uint64(k) for k in range(5)]))
    W = 8 + np.floor(u[0] * 57).astype(np.int64)
    nx = 256 + np.floor(u[1] * 1793).astype(np.int64)
    k = 10.0 ** (-4.0 + 2.0 * u[2])
    th = 20.0 + 20.0 * u[3]
    thr = 0.5 + 1.5 * u[4]
    return np.stack([W, nx, k, th, thr], axis=1).astype(np.float64)


def sweep_problem(row, instance: int, steps: int = 10_000) -> Problem:
    """One reactive capillary of the sweep: ny = W + 12, the capillary layout,
    D = 0.05, C0 = 1, adhesion from the contact angle, noise seed = instance."""
    W, nx, k, th, thr = row
    W, nx = int(W), int(nx)
    return capillary_problem(nx, W + 12, W, seed=int(instance), k_r=float(k),
                             threshold=float(thr), D=D_SOLUTE,
                             G_ads=adhesion_for_angle(float(th)), steps=steps,
                             name=f"sweep capillary {nx}x{W + 12} W={W}")


# --------------------------------------------------------------------------
# Surrogate of the sweep
# --------------------------------------------------------------------------
MLP_SIZES = (5, 256, 256, 256, 65)
MLP_NPARAMS = sum(a * b + b for a, b in zip(MLP_SIZES[:-1], MLP_SIZES[1:]))  # 149,825


def capillary_length(nx: int) -> int:
    """L = x_out - x_in of the capillary layout (x_in = nx // 3, x_out = nx - 32)."""
    return int(nx) - 32 - int(nx) // 3


def surrogate_box():
    """Normalisation / validity box of the surrogate inputs (W, L, k_r, theta,
    threshold), i.e. the range of the sweep sampler."""
    lo = np.array([8.0, capillary_length(256), 1e-4, 20.0, 0.5])
    hi = np.array([64.0, capillary_length(2048), 1e-2, 40.0, 2.0])
    return lo, hi


def surrogate_inputs(rows: np.ndarray) -> np.ndarray:
    """Sweep rows (W, nx, k_r, theta, threshold) -> surrogate inputs
    (W, L, k_r, theta, threshold)."""
    x = np.array(rows, dtype=np.float64).copy()
    x[:, 1] = [capillary_length(v) for v in x[:, 1]]
    return x


def mlp_init_params(seed: int) -> np.ndarray:
    """He-uniform weights U(-sqrt(6/fan_in), +sqrt(6/fan_in)) from the seeded
    SplitMix64 stream (one counter per weight, in packed order), zero biases.
    Packed order: W1 [256 x 5], b1, W2, b2, W3, b3, W4 [65 x 256], b4."""
    out = np.zeros(MLP_NPARAMS)
    off = 0
    ctr = 0
    for fan_in, fan_out in zip(MLP_SIZES[:-1], MLP_SIZES[1:]):
        nw = fan_in * fan_out
        u = uniform53(seed, np.arange(ctr, ctr + nw, dtype=np.uint64))
        ctr += nw
        a = np.sqrt(6.0 / fan_in)
        out[off:off + nw] = (2.0 * u - 1.0) * a
        off += nw + fan_out
    return out
