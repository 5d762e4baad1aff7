"""Pins of the FP64 surrogate MLP oracle: finite-difference gradients, the
closed-form first Adam step, a hand-wired network with a known output, and
the gradient's magnitude scale (an upper bound of every entry, equal to the
gradient when no sign can cancel)."""

import numpy as np

from oracle import mlp_oracle as M
from paper_1309_6726_amd import inputs


def _data(n, seed):
    rng = np.random.default_rng(seed)
    lo, hi = inputs.surrogate_box()
    x = lo + (hi - lo) * rng.uniform(size=(n, 5))
    x[:, 2] = 10 ** rng.uniform(-4, -2, n)
    t = rng.uniform(0, 1, (n, 65))
    return x, t, lo, hi


def test_gradients_match_central_differences():
    x, t, lo, hi = _data(7, 0)
    p = inputs.mlp_init_params(3) * 0.5
    p[1280:1280 + 256] = 0.05          # non-zero first biases
    w = np.linspace(0.5, 2.0, 65)
    _, g = M.loss_and_grad(p, x, t, lo, hi, w)
    rng = np.random.default_rng(1)
    idx = rng.choice(p.size, 60, replace=False)
    h = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        num = (M.loss_and_grad(pp, x, t, lo, hi, w)[0] - M.loss_and_grad(pm, x, t, lo, hi, w)[0]) / (2 * h)
        assert abs(num - g[i]) <= 1e-7 * max(1.0, abs(g[i])) + 1e-9, (i, num, g[i])


def test_first_adam_step_closed_form():
    rng = np.random.default_rng(2)
    p = rng.normal(size=50)
    g = rng.normal(size=50)
    p1, m, v = M.adam_step(p, np.zeros(50), np.zeros(50), g, 1, 1e-3)
    # bias-corrected moments equal g and g^2 after one step
    assert np.allclose(p1, p - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)


def test_hand_wired_network_reproduces_normalised_inputs():
    """W1 = [I5; 0], W2 = W3 = identity on the first 5 units, W4 row j picks
    unit j mod 5; with inputs normalised to (0, 1] the ReLUs pass them, so
    y_j = x'_(j mod 5) with x' = 2 (x - lo)/(hi - lo) - 1 (log10 for k_r)."""
    lo, hi = inputs.surrogate_box()
    x = np.array([[40.0, 1000.0, 3e-3, 35.0, 1.5], [60.0, 1300.0, 8e-3, 39.0, 1.9]])
    p = np.zeros(inputs.MLP_NPARAMS)
    layers = M.unpack(p)
    for k, (W, b) in enumerate(layers):
        for j in range(W.shape[0]):
            if k < 3 and j < 5:
                W[j, j] = 1.0
            elif k == 3:
                W[j, j % 5] = 1.0
    y, _ = M.forward(p, x, lo, hi)
    xn = np.array(x)
    xn[:, 2] = np.log10(xn[:, 2])
    l2, h2 = lo.copy(), hi.copy()
    l2[2], h2[2] = np.log10(lo[2]), np.log10(hi[2])
    expect = 2 * (xn - l2) / (h2 - l2) - 1
    assert (expect > 0).all()
    assert np.allclose(y, expect[:, np.arange(65) % 5], rtol=0, atol=1e-15)
    # the packed layout is the documented one: W1 first, then b1, ...
    assert layers[0][0].shape == (256, 5) and layers[3][0].shape == (65, 256)
    assert inputs.MLP_NPARAMS == 149825


def test_grad_error_scale_bounds_and_equality_case():
    """The scale bounds every gradient entry in magnitude; when every weight,
    bias and normalised input is positive and the targets are zero, no product
    changes sign, no ReLU cuts, and dL/dy = 2 w y / (rows sum w) = 2 w (|y| +
    |t|) / (rows sum w), so the scale equals the gradient itself."""
    x, t, lo, hi = _data(9, 3)
    w = np.linspace(0.5, 2.0, 65)
    for seed in (4, 5):
        p = inputs.mlp_init_params(seed)
        _, g = M.loss_and_grad(p, x, t, lo, hi, w)
        E = M.grad_error_scale(p, x, t, lo, hi, w)
        assert (E >= np.abs(g) * (1 - 1e-12)).all()
        assert (E > 0).mean() > 0.99
    rng = np.random.default_rng(6)
    p = np.abs(inputs.mlp_init_params(7)) + 1e-3
    xp = hi - (hi - lo) * rng.uniform(0.05, 0.45, size=(9, 5))  # normalised inputs in (0, 1)
    xp[:, 2] = 10 ** (np.log10(hi[2]) - rng.uniform(0.05, 0.45, 9) * (np.log10(hi[2]) - np.log10(lo[2])))
    assert (M.normalise(xp, lo, hi) > 0).all()
    t0 = np.zeros((9, 65))
    _, g = M.loss_and_grad(p, xp, t0, lo, hi, w)
    E = M.grad_error_scale(p, xp, t0, lo, hi, w)
    assert (g > 0).all()
    assert np.allclose(E, g, rtol=1e-12, atol=0)
