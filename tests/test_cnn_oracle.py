"""Pins of the CNN-surrogate oracle: a brute-force loop convolution, periodic
translation equivariance, finite-difference gradients, the closed form of
Adam under a constant gradient, and round-to-nearest-even bfloat16."""
import numpy as np
import pytest
import torch

from oracle import cnn
from paper_0901_3293_amd import inputs


def brute_conv(x, W, b):
    ci, nz, ny, nx = x.shape
    co = W.shape[0]
    y = np.zeros((co, nz, ny, nx))
    for o in range(co):
        for z in range(nz):
            for yy in range(ny):
                for xx in range(nx):
                    s = b[o]
                    for i in range(ci):
                        for kz in range(3):
                            for ky in range(3):
                                for kx in range(3):
                                    s += W[o, i, kz, ky, kx] * x[i, (z + kz - 1) % nz, (yy + ky - 1) % ny,
                                                                 (xx + kx - 1) % nx]
                    y[o, z, yy, xx] = s
    return y


def test_conv_matches_brute_force():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(2, 5, 3, 4))
    W = rng.normal(size=(3, 2, 3, 3, 3))
    b = rng.normal(size=3)
    assert np.abs(cnn.conv(x, W, b).numpy() - brute_conv(x, W, b)).max() < 1e-12


def test_conv_sites_matches_conv():
    rng = np.random.default_rng(5)
    x = rng.normal(size=(3, 5, 4, 6))
    W = rng.normal(size=(2, 3, 3, 3, 3))
    b = rng.normal(size=2)
    full = cnn.conv(x, W, b).numpy()
    sites = np.array([(0, 0, 0), (4, 3, 5), (2, 1, 3), (4, 0, 5)])
    got = cnn.conv_sites(x, W, b, sites)
    want = np.stack([full[:, z, y, xx] for z, y, xx in sites])
    assert np.abs(got - want).max() < 1e-12


def test_conv_periodic_translation_equivariance():
    rng = np.random.default_rng(1)
    x = torch.tensor(rng.normal(size=(4, 6, 5, 7)))
    W = torch.tensor(rng.normal(size=(3, 4, 3, 3, 3)))
    y = cnn.conv(x, W)
    sh = (2, -1, 3)
    ys = cnn.conv(torch.roll(x, sh, dims=(1, 2, 3)), W)
    assert torch.abs(ys - torch.roll(y, sh, dims=(1, 2, 3))).max() < 1e-12


def test_bf16_round_to_nearest_even():
    e = 2.0 ** -8
    vals = {1.0 + e: 1.0,                       # tie -> even mantissa (1.0)
            1.0 + 1.5 * e: 1.0 + 2 * e,         # above the tie
            1.0 + 2 * e + e: 1.0 + 4 * e,       # tie, odd lower neighbour -> up
            -1.0 - e: -1.0}
    for v, want in vals.items():
        assert float(cnn.bf16(torch.tensor(v, dtype=torch.float64))) == want


def test_param_count():
    assert cnn.param_count() == 18 * 32 * 27 + 32 + 2 * (32 * 32 * 27 + 32) + 32 * 5 * 27 + 5 == 75269


def test_backward_matches_finite_differences():
    """Gradient of the MSE loss (no rounding) against central differences on
    a random subset of parameters of every layer."""
    rng = np.random.default_rng(2)
    p = inputs.cnn_params(seed=3).astype(np.float64)
    p += rng.normal(0, 0.01, size=p.size)  # non-zero biases too
    x = rng.normal(size=(18, 4, 4, 4))
    t = rng.normal(size=(5, 4, 4, 4))
    acts, z = cnn.forward(p, x, rounding=False)
    g = cnn.backward(p, acts, z, t, rounding=False).numpy()

    def loss(q):
        _, zz = cnn.forward(q, x, rounding=False)
        return cnn.mse(zz, t)

    starts = np.cumsum([0] + [co * ci * 27 + co for co, ci, *_ in cnn.layer_shapes()])
    idx = []
    for l in range(4):
        idx += list(rng.integers(starts[l], starts[l + 1], size=6))
    h = 1e-6
    for i in idx:
        q1 = p.copy()
        q1[i] += h
        q2 = p.copy()
        q2[i] -= h
        fd = (loss(q1) - loss(q2)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g).max()), (i, fd, g[i])


def test_adam_constant_gradient_closed_form():
    """With a constant gradient the bias-corrected moments are exact, so every
    step moves each parameter by lr * g / (|g| + eps)."""
    g = np.array([0.3, -2.0, 1e-3])
    p = np.zeros(3)
    m = np.zeros(3)
    v = np.zeros(3)
    lr = 1e-2
    for t in range(1, 6):
        p_new, m, v = cnn.adam(p, g, m, v, t, lr)
        assert np.allclose(p_new - p, -lr * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
        p = p_new
