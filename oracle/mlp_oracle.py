"""FP64 reference of the surrogate MLP (5 -> 256 -> 256 -> 256 -> 65, ReLU).

TEST INFRASTRUCTURE ONLY: used by the tests to check the HIP forward,
backward and Adam kernels.  Plain numpy, written for reading.

Packed parameter order: W1 [256 x 5], b1, W2 [256 x 256], b2, W3, b3,
W4 [65 x 256], b4.  Inputs are normalised to [-1, 1] over the box [lo, hi]
(log10 for the reaction rate, column 2).  Loss: weighted mean squared error
sum_rows sum_j w_j (y - t)^2 / (rows * sum_j w_j).  Adam: beta1 0.9,
beta2 0.999, eps 1e-8, bias-corrected moments.
"""

from __future__ import annotations

import numpy as np

SIZES = (5, 256, 256, 256, 65)


def unpack(p):
    layers = []
    off = 0
    for fi, fo in zip(SIZES[:-1], SIZES[1:]):
        W = p[off:off + fi * fo].reshape(fo, fi)
        off += fi * fo
        b = p[off:off + fo]
        off += fo
        layers.append((W, b))
    return layers


def normalise(x, lo, hi):
    x = np.array(x, dtype=np.float64)
    lo = np.array(lo, dtype=np.float64).copy()
    hi = np.array(hi, dtype=np.float64).copy()
    x[:, 2] = np.log10(x[:, 2])
    lo[2], hi[2] = np.log10(lo[2]), np.log10(hi[2])
    return 2.0 * (x - lo) / (hi - lo) - 1.0


def forward(p, x, lo, hi):
    a = normalise(x, lo, hi)
    acts = [a]
    layers = unpack(np.asarray(p, dtype=np.float64))
    for k, (W, b) in enumerate(layers):
        z = a @ W.T + b
        a = np.maximum(z, 0.0) if k < len(layers) - 1 else z
        acts.append(a)
    return a, acts


def loss_and_grad(p, x, t, lo, hi, w=None):
    y, acts = forward(p, x, lo, hi)
    rows = y.shape[0]
    w = np.ones(SIZES[-1]) if w is None else np.asarray(w, dtype=np.float64)
    scale = 1.0 / (rows * w.sum())
    diff = y - t
    loss = float((w * diff * diff).sum() * scale)
    d = 2.0 * w * diff * scale
    layers = unpack(np.asarray(p, dtype=np.float64))
    grads = [None] * len(layers)
    for k in range(len(layers) - 1, -1, -1):
        W, _ = layers[k]
        grads[k] = (d.T @ acts[k], d.sum(axis=0))
        if k > 0:
            d = (d @ W) * (acts[k] > 0)
    g = np.concatenate([np.concatenate([gw.ravel(), gb]) for gw, gb in grads])
    return loss, g


def grad_error_scale(p, x, t, lo, hi, w=None):
    """Element-wise magnitude scale of the packed gradient: the gradient
    computation of loss_and_grad with every quantity replaced by a bound on its
    magnitude.  The forward pass uses |W| and |b| and no ReLU cut
    (|relu(z)| <= |z| <= |W| |a| + |b|); the output gradient uses
    2 w (|y| + |t|) / (rows sum w) >= |dL/dy|; deltas pass back through |W|
    and every unit.  An entry is thus at least the sum of the magnitudes of
    all products that make up that gradient entry (and of those that would,
    were a ReLU decided the other way), so a computation whose every product
    carries a relative error of at most u errs on it by at most
    (products in the chain) * u times this scale, to first order."""
    a = np.abs(normalise(x, lo, hi))
    acts = [a]
    layers = [(np.abs(W), np.abs(b)) for W, b in unpack(np.asarray(p, dtype=np.float64))]
    for W, b in layers:
        a = a @ W.T + b
        acts.append(a)
    rows = a.shape[0]
    w = np.ones(SIZES[-1]) if w is None else np.asarray(w, dtype=np.float64)
    scale = 1.0 / (rows * w.sum())
    d = 2.0 * w * (a + np.abs(t)) * scale
    grads = [None] * len(layers)
    for k in range(len(layers) - 1, -1, -1):
        W, _ = layers[k]
        grads[k] = (d.T @ acts[k], d.sum(axis=0))
        if k > 0:
            d = d @ W
    return np.concatenate([np.concatenate([gw.ravel(), gb]) for gw, gb in grads])


def adam_step(p, m, v, g, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
