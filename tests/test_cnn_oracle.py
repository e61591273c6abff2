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


# ---------------------------------------------------------------- the jump
# Pins of standardise / increment / jump (the surrogate jump as defined for
# this build: extrapolation base d1 + beta s2 plus the de-standardised network
# output; the paper defines no network).  Special cases whose value is fixed
# without the network: a zero network, a network that is a constant (its last
# bias), and a network that passes one standardised input channel through.


def _field(rng, c, shape=(4, 3, 5)):
    return rng.normal(size=(c,) + shape)


def _norm(rng, beta):
    norm = np.zeros(cnn.NORM_SIZE)
    norm[cnn.IN_MEAN:cnn.IN_MEAN + cnn.NIN] = rng.normal(size=cnn.NIN)
    norm[cnn.IN_STD:cnn.IN_STD + cnn.NIN] = rng.uniform(0.5, 2.0, size=cnn.NIN)
    norm[cnn.OUT_MEAN:cnn.OUT_MEAN + 5] = rng.normal(size=5) * 1e-3
    norm[cnn.OUT_STD:cnn.OUT_STD + 5] = rng.uniform(0.5, 2.0, size=5) * 1e-2
    norm[cnn.BETA] = beta
    return norm


def _state(rng):
    return _field(rng, 5), _field(rng, 3) * 1e-3, _field(rng, 5) * 1e-2, _field(rng, 5) * 1e-3


@pytest.mark.parametrize("beta", [0.0, 1.0, 0.5])
def test_increment_zero_network_is_the_extrapolation(beta):
    """All weights and biases zero and a zero target mean: the network adds
    nothing and the increment is the extrapolation d1 + beta s2 exactly."""
    rng = np.random.default_rng(11)
    norm = _norm(rng, beta)
    norm[cnn.OUT_MEAN:cnn.OUT_MEAN + 5] = 0.0
    Q, u, d1, s2 = _state(rng)
    got = cnn.increment(np.zeros(cnn.param_count()), norm, Q, u, d1, s2)
    assert np.array_equal(got, d1 + beta * s2)


def _last_bias_index(c):
    return cnn.param_count() - 5 + c


@pytest.mark.parametrize("c", [0, 3])
def test_increment_last_bias_destandardised_on_its_channel(c):
    """Zero weights and one non-zero bias b_c of the last layer: the network
    output is b_c on channel c and 0 elsewhere, so the increment is
    d1 + beta s2 + b_c std_c + mean_c on channel c and d1 + beta s2 + mean_c'
    on every other channel c' (de-standardisation with the target block)."""
    rng = np.random.default_rng(12 + c)
    beta = 1.0
    norm = _norm(rng, beta)
    p = np.zeros(cnn.param_count())
    p[_last_bias_index(c)] = 0.75
    Q, u, d1, s2 = _state(rng)
    got = cnn.increment(p, norm, Q, u, d1, s2)
    mean = norm[cnn.OUT_MEAN:cnn.OUT_MEAN + 5]
    std = norm[cnn.OUT_STD:cnn.OUT_STD + 5]
    for cc in range(5):
        want = d1[cc] + beta * s2[cc] + mean[cc] + (0.75 * std[cc] if cc == c else 0.0)
        assert np.abs(got[cc] - want).max() <= 1e-15, cc


def test_standardise_own_statistics_give_zero_mean_unit_std():
    """A field standardised with its own per-channel mean and standard
    deviation has mean 0 and standard deviation 1 on every channel (FP32)."""
    rng = np.random.default_rng(13)
    x = rng.normal(size=(cnn.NIN, 6, 5, 4)) * rng.uniform(0.1, 5.0, size=(cnn.NIN, 1, 1, 1)) \
        + rng.normal(size=(cnn.NIN, 1, 1, 1)) * 3
    flat = x.reshape(cnn.NIN, -1)
    norm = np.zeros(cnn.NORM_SIZE)
    norm[cnn.IN_MEAN:cnn.IN_MEAN + cnn.NIN] = flat.mean(axis=1)
    norm[cnn.IN_STD:cnn.IN_STD + cnn.NIN] = flat.std(axis=1)
    xs = cnn.standardise(x, norm).reshape(cnn.NIN, -1).astype(np.float64)
    assert np.abs(xs.mean(axis=1)).max() <= 1e-5
    assert np.abs(xs.std(axis=1) - 1.0).max() <= 1e-5


@pytest.mark.parametrize("ch", [2, 6, 9, 14])
def test_increment_passes_one_standardised_channel(ch):
    """A network that passes input channel ch to output channel 0 (centre tap
    1 through every layer, all else zero) outputs relu of that standardised
    input (rounded to bfloat16); the input order is Q (0-4), u (5-7), d1
    (8-12), s2 (13-17)."""
    rng = np.random.default_rng(20 + ch)
    norm = _norm(rng, 0.0)
    Q, u, d1, s2 = _state(rng)
    p = np.zeros(cnn.param_count())
    k = 0
    for l, (co, ci, *_) in enumerate(cnn.layer_shapes()):
        W = np.zeros((co, ci, 3, 3, 3))
        W[0, ch if l == 0 else 0, 1, 1, 1] = 1.0
        p[k:k + W.size] = W.ravel()
        k += W.size + co
    got = cnn.increment(p, norm, Q, u, d1, s2)
    raw = np.concatenate([Q, u, d1, s2])[ch]
    xs = (raw.astype(np.float32) - np.float32(norm[cnn.IN_MEAN + ch])) / np.float32(norm[cnn.IN_STD + ch])
    net0 = cnn.bf16(torch.tensor(np.maximum(xs, 0).astype(np.float64))).numpy()
    mean = norm[cnn.OUT_MEAN:cnn.OUT_MEAN + 5]
    std = norm[cnn.OUT_STD:cnn.OUT_STD + 5]
    assert np.abs(got[0] - (d1[0] + net0 * std[0] + mean[0])).max() <= 1e-15
    for cc in range(1, 5):
        assert np.abs(got[cc] - (d1[cc] + mean[cc])).max() <= 1e-15


def test_jump_advances_state_and_history():
    """One jump: Q' = Q + dq, d1' = dq, s2' = dq - d1, with dq fixed in closed
    form by a constant network (last bias) on the quadratic base."""
    rng = np.random.default_rng(30)
    norm = _norm(rng, 1.0)
    p = np.zeros(cnn.param_count())
    p[_last_bias_index(1)] = -0.5
    Q, u, d1, s2 = _state(rng)
    mean = norm[cnn.OUT_MEAN:cnn.OUT_MEAN + 5][:, None, None, None]
    std = norm[cnn.OUT_STD:cnn.OUT_STD + 5][:, None, None, None]
    net = np.zeros((5, 1, 1, 1))
    net[1] = -0.5
    dq = d1 + s2 + net * std + mean
    Qn, d1n, s2n = cnn.jump(p, norm, Q, u, d1, s2)
    assert np.abs(Qn - (Q + dq)).max() <= 1e-15
    assert np.abs(d1n - dq).max() <= 1e-15
    assert np.abs(s2n - (dq - d1)).max() <= 1e-15
    # the history of two consecutive jumps of a zero network on the linear
    # base: the increment repeats and its change vanishes
    z = np.zeros(cnn.param_count())
    nz = _norm(rng, 0.0)
    nz[cnn.OUT_MEAN:cnn.OUT_MEAN + 5] = 0.0
    Q1, a1, b1 = cnn.jump(z, nz, Q, u, d1, s2)
    Q2, a2, b2 = cnn.jump(z, nz, Q1, u, a1, b1)
    assert np.array_equal(a2, d1) and not np.any(b2) and np.abs(Q2 - (Q + 2 * d1)).max() <= 1e-15


def _shift(a, d):
    """a[..., s + d] on the periodic lattice (d = (dz, dy, dx))."""
    return np.roll(a, shift=(-d[0], -d[1], -d[2]), axis=(1, 2, 3))


def test_backward_with_rounding_matches_direct_sums():
    """backward(rounding=True) against the weight, bias and data gradients
    written as direct FP64 sums over sites and taps of the bfloat16-rounded
    operands: dz of the loss rounded, weights rounded, the data gradient of
    each layer masked by the ReLU of its input and rounded again (4^3
    lattice, random network and target)."""
    rng = np.random.default_rng(40)
    p = inputs.cnn_params(seed=5).astype(np.float64) + rng.normal(0, 0.01, size=cnn.param_count())
    x = rng.normal(size=(18, 4, 4, 4))
    t = rng.normal(size=(5, 4, 4, 4))
    acts, z = cnn.forward(p, x, rounding=True)
    got = cnn.backward(p, acts, z, t, rounding=True).numpy()

    def r(a):
        return cnn.bf16(torch.tensor(np.asarray(a, dtype=np.float64))).numpy()

    layers = [(W.numpy(), b.numpy()) for W, b in cnn.unflatten(p)]
    n = z.numel()
    dz = r(2.0 * (z.numpy() - t) / n)
    want = [None] * 4
    taps = [(kz, ky, kx) for kz in range(3) for ky in range(3) for kx in range(3)]
    for l in range(3, -1, -1):
        a = np.asarray(acts[l], dtype=np.float64)
        Wr = r(layers[l][0])
        co, ci = Wr.shape[:2]
        dW = np.zeros_like(Wr)
        dx = np.zeros_like(a)
        for kz, ky, kx in taps:
            d = (kz - 1, ky - 1, kx - 1)
            src = _shift(a, d)  # the input each output site reads through this tap
            dW[:, :, kz, ky, kx] = dz.reshape(co, -1) @ src.reshape(ci, -1).T
            # each output site s sends W dz(s) back to the input site s + d
            back = np.tensordot(Wr[:, :, kz, ky, kx], dz, axes=([0], [0]))
            dx += np.roll(back, shift=d, axis=(1, 2, 3))
        want[l] = np.concatenate([dW.ravel(), dz.reshape(co, -1).sum(axis=1)])
        if l > 0:
            dz = r(dx * (a > 0))
    want = np.concatenate(want)
    scale = np.abs(want).max()
    assert np.abs(got - want).max() <= 1e-12 * scale
