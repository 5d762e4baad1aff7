"""Learned surrogate of the capillary sweep, trained on batched LB runs.

The network (5 -> 256 -> 256 -> 256 -> 65) is trained and evaluated by the
HIP kernels behind surr_* (include/lbm.h); this module marshals arguments and
drives the pipeline:

  * data: reactive capillary runs from the sweep sampler advanced by the
    batched lattice Boltzmann path (front z(t_j) at t_j = ceil(j T / 64) and
    the pore-closure step);
  * targets: z(t_j) / S and closure / T (1 when not closed), where S is the
    travel of the linear Washburn law, Eq. (1), at long times,
    v T = gamma cos(theta) W T / (6 mu (L + L_e)), capped at L, plus 1 lu:
    this makes every trajectory O(1) whatever its speed, so the loss tracks the
    front error relative to the travel; the network learns the deviation from
    the law (retardation by surface growth, pore closure, breakthrough);
  * confidence: an ensemble of networks trained from different seeds answers
    with its mean; a query goes to the lattice Boltzmann model when the
    predicted travel is small or the members disagree (spread relative to the
    travel), with both gates chosen on held-back training runs;
  * queries outside the training box go to the lattice Boltzmann model.
"""

from __future__ import annotations

import ctypes as C
import math
import time

import numpy as np

from . import inputs, lbm, sweep

GAMMA = 0.0761          # surface tension at G = 1.6 (Laplace calibration)
MU = 1.0614 / 6.0       # dynamic viscosity: total density x (tau - 1/2) / 3
ENTRANCE = 1.35         # entrance length in units of the width (Washburn runs)
NSLOTS = 64


def washburn_scale(x: np.ndarray, T: int) -> np.ndarray:
    """S = min(v T, L) + 1 with v = gamma cos(theta) W / (6 mu (L + 1.35 W))."""
    W, L, th = x[:, 0], x[:, 1], x[:, 3]
    v = GAMMA * np.cos(np.radians(th)) * W / (6.0 * MU * (L + ENTRANCE * W))
    return np.minimum(v * T, L) + 1.0


def make_targets(x, fronts, closure, T):
    S = washburn_scale(x, T)
    z = fronts / S[:, None]
    c = np.where(closure >= 0, closure / float(T), 1.0)
    return np.concatenate([z, c[:, None]], axis=1).astype(np.float32)


def decode(x, y, T):
    """Network outputs -> (fronts in lattice units, closure step or -1)."""
    S = washburn_scale(x, T)
    fronts = y[:, :NSLOTS] * S[:, None]
    L = x[:, 1]
    fronts = np.clip(fronts, 0.0, L[:, None])
    c = y[:, NSLOTS]
    closure = np.where(c < 0.995, np.round(np.clip(c, 0, 1) * T), -1).astype(np.int64)
    return fronts, closure


def front_error(pred, true):
    """Per run: RMS_j |z_hat_j - z_j| / max(z(T) - z(0), 1 lu), z(0) = 0."""
    travel = np.maximum(true[:, -1], 1.0)
    return np.sqrt(np.mean((pred - true) ** 2, axis=1)) / travel


def in_box(x, lo, hi):
    return np.all((x >= lo - 1e-9 * np.abs(lo)) & (x <= hi + 1e-9 * np.abs(hi)), axis=1)


class Surrogate:
    def __init__(self, max_batch=256, max_data=8192, *, device="cuda:0", stream=None):
        import torch
        self.lo, self.hi = inputs.surrogate_box()
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        L = lbm.lib()
        n = C.c_size_t(0)
        lbm.check(L.surr_workspace_bytes(int(max_batch), int(max_data), C.byref(n)))
        self.workspace = torch.empty(n.value + 256, dtype=torch.uint8, device=self.device)
        ws = (self.workspace.data_ptr() + 255) // 256 * 256
        lo = np.ascontiguousarray(self.lo, dtype=np.float64)
        hi = np.ascontiguousarray(self.hi, dtype=np.float64)
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            lbm.check(L.surr_init(lo.ctypes.data, hi.ctypes.data, int(max_batch), int(max_data),
                                  C.c_void_p(self.stream.cuda_stream), C.c_void_p(ws), n.value,
                                  C.byref(h)))
        self.h = h
        self.max_batch = int(max_batch)

    def close(self):
        if getattr(self, "h", None):
            lbm.lib().surr_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, p):
        a = np.ascontiguousarray(p, dtype=np.float32)
        assert a.size == inputs.MLP_NPARAMS
        lbm.check(lbm.lib().surr_set_params(self.h, a.ctypes.data))

    def params(self):
        a = np.zeros(inputs.MLP_NPARAMS, dtype=np.float32)
        lbm.check(lbm.lib().surr_get_params(self.h, a.ctypes.data))
        return a

    def set_loss_weights(self, w):
        a = np.ascontiguousarray(w, dtype=np.float32)
        lbm.check(lbm.lib().surr_set_loss_weights(self.h, a.ctypes.data))

    def set_data(self, x, y, row_weights=None):
        x = np.ascontiguousarray(x, dtype=np.float32)
        y = np.ascontiguousarray(y, dtype=np.float32)
        w = None if row_weights is None else np.ascontiguousarray(row_weights, dtype=np.float32)
        self._n = x.shape[0]
        lbm.check(lbm.lib().surr_set_data(self.h, x.ctypes.data, y.ctypes.data,
                                          None if w is None else w.ctypes.data, self._n))

    def train_epoch(self, perm, batch, lr):
        p = np.ascontiguousarray(perm, dtype=np.int32)
        loss = C.c_double(0)
        lbm.check(lbm.lib().surr_train_epoch(self.h, p.ctypes.data, int(batch), float(lr),
                                             C.byref(loss)))
        return loss.value

    def gradients(self, x, y):
        x = np.ascontiguousarray(x, dtype=np.float32)
        y = np.ascontiguousarray(y, dtype=np.float32)
        g = np.zeros(inputs.MLP_NPARAMS, dtype=np.float32)
        loss = C.c_double(0)
        lbm.check(lbm.lib().surr_gradients(self.h, x.ctypes.data, y.ctypes.data, x.shape[0],
                                           g.ctypes.data, C.byref(loss)))
        return loss.value, g

    def predict(self, x):
        x = np.ascontiguousarray(x, dtype=np.float32)
        y = np.zeros((x.shape[0], inputs.MLP_SIZES[-1]), dtype=np.float32)
        lbm.check(lbm.lib().surr_predict(self.h, x.ctypes.data, x.shape[0], y.ctypes.data))
        return y

    def predict_noalloc(self, x_dev, y_dev, stream=None):
        """surr_predict_noalloc: x_dev [n x 5] and y_dev [n x 65] are contiguous
        FP32 torch tensors on the handle's GPU; queued on `stream` (default:
        the handle's), nothing allocated, no synchronisation."""
        import torch
        assert x_dev.dtype == torch.float32 and y_dev.dtype == torch.float32
        assert x_dev.is_contiguous() and y_dev.is_contiguous()
        n = x_dev.shape[0]
        assert x_dev.shape == (n, inputs.MLP_SIZES[0]) and y_dev.shape == (n, inputs.MLP_SIZES[-1])
        st = self.stream if stream is None else stream
        lbm.check(lbm.lib().surr_predict_noalloc(self.h, C.c_void_p(x_dev.data_ptr()), n,
                                                 C.c_void_p(y_dev.data_ptr()),
                                                 C.c_void_p(st.cuda_stream)))


class Ensemble:
    """K networks trained from different seeds (initial weights and minibatch
    order).  The answer is the mean of the members' outputs; the spread of
    their decoded fronts measures how far the ensemble can be trusted."""

    def __init__(self, k: int = 3, **kw):
        self.members = [Surrogate(**kw) for _ in range(k)]
        self.lo, self.hi = self.members[0].lo, self.members[0].hi

    def train(self, x, y, *, seed: int = 0, **kw):
        """Member i is trained from seed + i; returns the loss histories."""
        return [train(net, x, y, seed=seed + i, **kw) for i, net in enumerate(self.members)]

    def predict(self, x):
        return np.mean([net.predict(x).astype(np.float64) for net in self.members], axis=0)

    def predict_with_spread(self, x, T: int):
        """(mean outputs, relative spread): the largest over sample times of the
        members' standard deviation of z(t_j), over max(predicted travel, 1 lu)."""
        ys = np.stack([net.predict(x).astype(np.float64) for net in self.members])
        y = ys.mean(axis=0)
        fr = np.stack([decode(x, yk, T)[0] for yk in ys])
        mean_travel = decode(x, y, T)[0][:, -1]
        spread = fr.std(axis=0).max(axis=1) / np.maximum(mean_travel, 1.0)
        return y, spread

    def close(self):
        for net in self.members:
            net.close()


def generate(seed: int, n: int, T: int, *, chunk: int = 512, device="cuda:0", log=None):
    """n sweep runs (sampler seed) advanced by the batched LB path.
    Returns (rows, x, fronts, closure, seconds)."""
    rows = inputs.sweep_params(seed, n)
    fronts = np.zeros((n, NSLOTS))
    closure = np.zeros(n, dtype=np.int64)
    t0 = time.perf_counter()
    tile = None
    for s in range(0, n, chunk):
        probs = [inputs.sweep_problem(r, s + i, steps=T) for i, r in enumerate(rows[s:s + chunk])]
        f, c, sec, tile = sweep.run_batched(probs, T, NSLOTS, tile=tile, autotune=tile is None,
                                           device=device)
        fronts[s:s + len(probs)] = f
        closure[s:s + len(probs)] = c
        if log:
            log(f"  generated runs {s}..{s + len(probs) - 1} in {sec:.1f} s (tile {tile})")
    return rows, inputs.surrogate_inputs(rows), fronts, closure, time.perf_counter() - t0


def train(net: Surrogate, x, y, *, epochs=3000, batch=256, lr=2e-3, lr_min=2e-5, seed=0,
          log=None, log_every=500, weights=None):
    """Adam with a cosine learning-rate schedule; permutations from the seeded
    stream.  Returns the loss history (one value per logged epoch)."""
    net.set_params(inputs.mlp_init_params(seed))
    net.set_data(x, y, weights)
    n = x.shape[0]
    hist = []
    for e in range(epochs):
        key = inputs.uniform53(seed + 1000003 * (e + 1), np.arange(n, dtype=np.uint64))
        perm = np.argsort(key, kind="stable").astype(np.int32)
        rate = lr_min + 0.5 * (lr - lr_min) * (1 + math.cos(math.pi * e / max(1, epochs - 1)))
        loss = net.train_epoch(perm, batch, rate)
        if e % log_every == 0 or e == epochs - 1:
            hist.append((e, loss))
            if log:
                log(f"  epoch {e}: loss {loss:.3e} lr {rate:.2e}")
    return hist


def joint_gates(travel, spread, err, target=0.01, p95=0.02, min_frac=0.25):
    """The (travel gate, spread gate) pair that answers the most runs among
    those whose answered runs (predicted travel >= travel gate and relative
    spread <= spread gate) have mean front error <= target and a 95th
    percentile of the error <= p95, and make up at least min_frac of the runs.
    Travel gates are whole lattice units 0..100.  Returns (inf, -1.0) when no
    pair qualifies (every query then goes to the lattice Boltzmann model)."""
    travel, spread, err = (np.asarray(v, dtype=np.float64) for v in (travel, spread, err))
    n = len(err)
    need = int(math.ceil(min_frac * n))
    best, best_n = (float("inf"), -1.0), 0
    for z in np.arange(0.0, 101.0, 1.0):
        sel = np.nonzero(travel >= z)[0]
        if len(sel) < max(need, 1):
            break
        order = sel[np.argsort(spread[sel], kind="stable")]
        e = err[order]
        sp = spread[order]
        cmean = np.cumsum(e) / np.arange(1, len(e) + 1)
        for k in range(len(e), 0, -1):  # largest answered set first
            if k < need or k <= best_n:
                break
            if k < len(e) and sp[k] == sp[k - 1]:
                continue  # a gate at sp[k-1] would also admit run k
            if cmean[k - 1] <= target and np.quantile(e[:k], 0.95) <= p95:
                best, best_n = (float(z), float(sp[k - 1])), k
                break
    return best


def choose_gates(model, x, fronts, T, target=0.01, p95=0.02, min_frac=0.25):
    """Both gates of an ensemble from held-back runs whose lattice Boltzmann
    fronts are known (joint_gates on its predictions)."""
    y, spread = model.predict_with_spread(x, T)
    f, _ = decode(x, y, T)
    err = front_error(f, fronts)
    return joint_gates(f[:, -1], spread, err, target, p95, min_frac)


def answer(net, rows, T: int, gate, *, device="cuda:0"):
    """Sweep queries answered by the network (a Surrogate or an Ensemble) where
    it is in its box and confident, by the batched lattice Boltzmann model
    otherwise.  gate: minimum predicted travel z_hat(T) in lattice units, or
    for an ensemble (travel gate, spread gate).  Returns (fronts, closure,
    used_net mask, net_seconds, lb_seconds); lb_seconds covers building the
    fallback batch as well as running it."""
    x = inputs.surrogate_inputs(rows)
    ok = in_box(x, net.lo, net.hi)
    fronts = np.zeros((len(rows), NSLOTS))
    closure = np.zeros(len(rows), dtype=np.int64)
    use = np.zeros(len(rows), dtype=bool)
    g_travel, g_spread = (gate, None) if np.isscalar(gate) else gate
    t0 = time.perf_counter()
    if ok.any():
        if g_spread is None:
            y = net.predict(x[ok]).astype(np.float64)
            spread = np.zeros(int(ok.sum()))
        else:
            y, spread = net.predict_with_spread(x[ok], T)
        f, c = decode(x[ok], y, T)
        conf = f[:, -1] >= g_travel
        if g_spread is not None:
            conf &= spread <= g_spread
        idx = np.nonzero(ok)[0][conf]
        fronts[idx], closure[idx] = f[conf], c[conf]
        use[idx] = True
    net_sec = time.perf_counter() - t0
    lb_sec = 0.0
    rest = np.nonzero(~use)[0]
    if len(rest):
        probs = [inputs.sweep_problem(rows[i], int(i), steps=T) for i in rest]
        f, c, lb_sec, _ = sweep.run_batched(probs, T, NSLOTS, device=device)
        fronts[rest], closure[rest] = f, c
    return fronts, closure, use, net_sec, lb_sec


def out_of_range_rows(seed: int, n: int = 32):
    """Queries outside the training box: width 72..96 or reaction rate
    1.2e-2..5e-2 (the other inputs inside the box)."""
    base = inputs.sweep_params(seed, n)
    u = inputs.uniform53(seed + 7, np.arange(2 * n, dtype=np.uint64)).reshape(2, n)
    rows = base.copy()
    for i in range(n):
        if i % 2 == 0:
            rows[i, 0] = 72 + np.floor(u[0, i] * 25)
            rows[i, 1] = 256 + np.floor(u[1, i] * 512)
        else:
            rows[i, 2] = 1.2e-2 + u[0, i] * 3.8e-2
    return rows
