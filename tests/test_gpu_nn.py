"""Surrogate kernels against the CNN oracle, through the C-ABI.

Per layer, on the same bfloat16 operands: forward pre-activation, weight and
bias gradients and the backward-data convolution within 1e-5 relative of the
FP64 oracle (FP32 accumulation of at most 864 exact bf16 products).  Whole
network, teacher-forced: each layer of a full training step is checked on
the very operands the GPU passed it (hlbnn_grad_trace), so the output and
the gradient of every layer are held to the same 1e-5, and each bfloat16
activation or gradient the GPU hands on is within half an ulp of the
oracle's exact value.  Free-running (the oracle's own activations), the two
sides may round a few activations to different neighbours at ties; the
whole-network output and gradient are held to 1e-3 there, with the number of
such flips reported."""
import numpy as np
import pytest
import torch

from oracle import cnn
from paper_0901_3293_amd import inputs
from tests.hlbtest import rel, say

pytestmark = pytest.mark.gpu

CIP = (32, 32, 32, 32)
COP = (32, 32, 32, 16)
CI = (18, 32, 32, 32)
CO = (32, 32, 32, 5)


@pytest.fixture(scope="module")
def H():
    assert torch.cuda.is_available()
    from paper_0901_3293_amd import hlb

    return hlb


def to_bf16_bits(a):
    """float array -> bfloat16 bit patterns (RNE), same shape."""
    t = torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32)).to(torch.bfloat16)
    return t.view(torch.int16).numpy().view(np.uint16)


def channels_last(a, cpad):
    """[C][z][y][x] -> [N][cpad] (zero padded)."""
    C = a.shape[0]
    out = np.zeros((a[0].size, cpad))
    out[:, :C] = np.asarray(a).reshape(C, -1).T
    return out


def from_channels_last(a, C, shape):
    nx, ny, nz = shape
    return np.asarray(a)[:, :C].T.reshape(C, nz, ny, nx)


SHAPES = [(16, 8, 8), (20, 6, 9), (40, 20, 12)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("layer", [0, 1, 3])
def test_layer_forward(H, shape, layer):
    say("case: nn layer forward", shape, layer)
    rng = np.random.default_rng(10 + layer)
    net = H.Net(shape)
    p = inputs.cnn_params(seed=layer)
    p[-(5 + 1):] = 0
    p = (p + rng.normal(0, 0.02, size=p.size)).astype(np.float32)
    net.set_params(p)
    x = rng.normal(size=(CI[layer],) + shape[::-1])
    xb = to_bf16_bits(channels_last(x, CIP[layer]))
    z = net.layer_forward(layer, xb)
    W, b = cnn.unflatten(p)[layer]
    xr = cnn.bf16(torch.tensor(x))
    ref = cnn.conv(xr, cnn.bf16(W), b).numpy()
    got = from_channels_last(z, CO[layer], shape)
    e = rel(got, ref)
    say("rel err", e)
    assert e <= 1e-5


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("layer", [0, 2, 3])
def test_layer_backward(H, shape, layer):
    say("case: nn layer backward", shape, layer)
    rng = np.random.default_rng(20 + layer)
    net = H.Net(shape)
    p = (inputs.cnn_params(seed=5) + rng.normal(0, 0.02, size=cnn.param_count())).astype(np.float32)
    net.set_params(p)
    x = rng.normal(size=(CI[layer],) + shape[::-1])
    dz = rng.normal(size=(CO[layer],) + shape[::-1]) * 1e-3
    xb = to_bf16_bits(channels_last(x, CIP[layer]))
    dzb = to_bf16_bits(channels_last(dz, COP[layer]))
    dx, g = net.layer_backward(layer, xb, dzb)
    W, _ = cnn.unflatten(p)[layer]
    dW, db, dxr = cnn.layer_backward(cnn.bf16(torch.tensor(x)), cnn.bf16(torch.tensor(dz)), cnn.bf16(W))
    gref = torch.cat([dW.reshape(-1), db]).numpy()
    e_w = rel(g[:-CO[layer]], gref[:-CO[layer]])
    e_b = rel(g[-CO[layer]:], gref[-CO[layer]:])
    e_x = rel(from_channels_last(dx, CI[layer], shape), dxr.numpy())
    say("rel err dW, db, dx", e_w, e_b, e_x)
    assert e_w <= 1e-5 and e_b <= 1e-5 and e_x <= 1e-5


@pytest.mark.parametrize("layer", [1, 3])
def test_weight_gradient_full_size_sampled(H, layer):
    """Weight and bias gradient of one layer on the 96^3 lattice of the
    surrogate workload, where each block of the weight-gradient kernel
    accumulates several tiles: the whole bias gradient against the FP64 sum of
    the bfloat16 output gradient, and 64 sampled weight-gradient entries
    against direct FP64 sums over all sites (same bfloat16 operands; FP32
    accumulation, bar 1e-5 of the largest entry)."""
    shape = (96, 96, 96)
    say("case: weight gradient 96^3, layer", layer)
    nx, ny, nz = shape
    rng = np.random.default_rng(30 + layer)
    net = H.Net(shape)
    net.set_params(inputs.cnn_params(seed=5))
    x = rng.normal(size=(CI[layer],) + shape[::-1]).astype(np.float32)
    dz = (rng.normal(size=(CO[layer],) + shape[::-1]) * 1e-3).astype(np.float32)
    xb = to_bf16_bits(channels_last(x, CIP[layer]))
    dzb = to_bf16_bits(channels_last(dz, COP[layer]))
    _, g = net.layer_backward(layer, xb, dzb)
    xf = cnn.bf16(torch.tensor(x)).double().numpy()    # [ci][z][y][x]
    dzf = cnn.bf16(torch.tensor(dz)).double().numpy()  # [co][z][y][x]
    ci_n, co_n = CI[layer], CO[layer]
    db = dzf.reshape(co_n, -1).sum(1)
    gb = g[-co_n:]
    eb = np.abs(gb - db).max() / np.abs(db).max()
    gw = g[:-co_n].reshape(co_n, ci_n, 27)  # W[co][ci][tap], tap = kz*9 + ky*3 + kx
    ref, got = [], []
    for _ in range(64):
        co, ci, tap = int(rng.integers(co_n)), int(rng.integers(ci_n)), int(rng.integers(27))
        kz, ky, kx = tap // 9, (tap // 3) % 3, tap % 3
        shifted = np.roll(xf[ci], shift=(-(kz - 1), -(ky - 1), -(kx - 1)), axis=(0, 1, 2))  # X(s + off)
        ref.append(float((dzf[co] * shifted).sum()))
        got.append(float(gw[co, ci, tap]))
    ref, got = np.array(ref), np.array(got)
    ew = np.abs(got - ref).max() / np.abs(ref).max()
    say("rel err db, sampled dW", eb, ew)
    assert eb <= 1e-5 and ew <= 1e-5


def norm_block(x, dq, beta):
    """Standardisation block (47 floats) from one raw input x [18, ...] and
    target dq [5, ...]."""
    c = dq - x[8:13] - beta * x[13:18]
    v = np.zeros(cnn.NORM_SIZE)
    v[cnn.IN_MEAN:cnn.IN_MEAN + 18] = x.reshape(18, -1).mean(1)
    v[cnn.IN_STD:cnn.IN_STD + 18] = x.reshape(18, -1).std(1) + 1e-12
    v[cnn.OUT_MEAN:cnn.OUT_MEAN + 5] = c.reshape(5, -1).mean(1)
    v[cnn.OUT_STD:cnn.OUT_STD + 5] = c.reshape(5, -1).std(1) + 1e-12
    v[cnn.BETA] = beta
    return v.astype(np.float32)


def random_inputs(rng, shape):
    """Raw inputs with the scales of a solver state: Q ~ 0.1, u ~ 1e-4, d1 ~
    1e-3, s2 ~ 1e-5."""
    sc = np.array([0.1] * 5 + [1e-4] * 3 + [1e-3] * 5 + [1e-5] * 5)
    return rng.normal(size=(18,) + shape[::-1]) * sc[:, None, None, None]


def test_network_forward_and_training_step(H):
    """Whole network and one Adam step on a 24x12x16 lattice, extrapolation
    weight beta = 1, free-running (the oracle rounds its own activations).
    Bars: predicted increment within 5e-3 (max) of the network's share of it
    (the two sides round a few activations to different bfloat16 neighbours
    at ties, which moves the output by up to about 2e-3 of its scale; the
    teacher-forced test below holds every layer to 1e-5 instead); gradient
    within 1e-3 relative; loss within 1e-4; Adam update exactly the textbook
    step on the GPU's own gradient (1e-6)."""
    say("case: nn network forward + train step")
    shape = (24, 12, 16)
    rng = np.random.default_rng(3)
    net = H.Net(shape)
    p0 = (inputs.cnn_params(seed=7) + rng.normal(0, 0.01, size=cnn.param_count())).astype(np.float32)
    net.set_params(p0)
    x = random_inputs(rng, shape)
    dq = x[8:13] + x[13:18] + rng.normal(size=(5,) + shape[::-1]) * 1e-6
    norm = norm_block(x, dq, 1.0)
    net.set_norm(norm)
    xd = torch.tensor(x, dtype=torch.float32, device="cuda")
    dqd = torch.tensor(dq, dtype=torch.float32, device="cuda")
    out = net.predict(xd).cpu().numpy().astype(np.float64)
    x32 = x.astype(np.float32)
    ref = cnn.increment(p0, norm, x32[:5], x32[5:8], x32[8:13], x32[13:18])
    share = ref - x32[8:13].astype(np.float64) - x32[13:18].astype(np.float64)
    d = np.abs(out - ref)
    say("forward rel max, mean:", d.max() / np.abs(share).max(), d.mean() / np.abs(share).mean())
    assert d.max() / np.abs(share).max() <= 5e-3
    loss = net.train_step(xd, dqd, lr=1e-3)
    acts, z = cnn.forward(p0, cnn.standardise(x32, norm))
    c = dq.astype(np.float32) - x32[8:13] - np.float32(1.0) * x32[13:18]
    t = (c - norm[cnn.OUT_MEAN:cnn.OUT_MEAN + 5, None, None, None]) / norm[cnn.OUT_STD:cnn.OUT_STD + 5, None, None, None]
    loss_ref = cnn.mse(z, t)
    say("loss gpu, oracle:", loss, loss_ref)
    assert abs(loss - loss_ref) <= 1e-4 * loss_ref
    g = net.grads()
    gref = cnn.backward(p0, acts, z, t).numpy()
    eg = rel(g, gref)
    say("grad rel err", eg)
    assert eg <= 1e-3
    p1 = net.params()
    p_ref, _, _ = cnn.adam(p0, g, np.zeros_like(g), np.zeros_like(g), 1, 1e-3)
    assert np.abs(p1 - p_ref).max() <= 1e-6 * max(1.0, np.abs(p_ref).max())


def test_training_is_deterministic(H):
    say("case: nn training determinism")
    shape = (16, 8, 12)
    rng = np.random.default_rng(4)
    xh = random_inputs(rng, shape)
    dqh = xh[8:13] + rng.normal(size=(5,) + shape[::-1]) * 1e-5
    x = torch.tensor(xh, dtype=torch.float32, device="cuda")
    dq = torch.tensor(dqh, dtype=torch.float32, device="cuda")
    res = []
    for _ in range(2):
        net = H.Net(shape)
        net.set_params(inputs.cnn_params(seed=1))
        net.set_norm(norm_block(xh, dqh, 0.0))
        for _ in range(3):
            net.train_step(x, dq, 1e-3, want_loss=False)
        res.append(net.params())
    assert np.array_equal(res[0], res[1])


def bits_to_f64(bits):
    return torch.from_numpy(np.ascontiguousarray(bits).view(np.int16)).view(torch.bfloat16).to(torch.float64).numpy()


def handed_on(got, exact, zscale, name):
    """A bfloat16 value the GPU hands to the next layer against the oracle's
    exact FP64 value of the same quantity: within half an ulp of bfloat16
    (at most 2^-8 of the value: 8 significant bits) plus the FP32
    accumulation bar (2e-5 of the layer's scale).  Returns the number of entries that round to a different
    bfloat16 neighbour than the exact value does (ties split by rounding
    error)."""
    bound = 2.0 ** -8 * np.abs(exact) + 2e-5 * zscale
    bad = np.abs(got - exact) > bound
    assert not bad.any(), (name, int(bad.sum()), float(np.abs(got - exact).max()))
    return int((got != cnn.bf16(torch.tensor(exact)).numpy()).sum())


def test_network_teacher_forced(H):
    """One training step on a 24x12x16 lattice (beta = 1), every layer
    checked on the operands the GPU itself passed it: each layer's
    pre-activation from the GPU's bfloat16 input against the oracle's FP64
    convolution of that input (last layer: the FP32 output within 1e-5;
    hidden layers: the bfloat16 activation handed on within half an ulp);
    the loss gradient; each layer's weight and bias gradient from the GPU's
    input and output gradient within 1e-5 relative (so a 1% scale error in
    the weight-gradient kernel fails); each backward-data output handed on
    within half an ulp.  Then the whole network free-running against the
    oracle's own forward and backward within 1e-3, with the tie flips per
    layer reported."""
    say("case: nn teacher-forced network")
    shape = (24, 12, 16)
    nx, ny, nz = shape
    rng = np.random.default_rng(8)
    net = H.Net(shape)
    p0 = (inputs.cnn_params(seed=9) + rng.normal(0, 0.01, size=cnn.param_count())).astype(np.float32)
    net.set_params(p0)
    x = random_inputs(rng, shape)
    dq = x[8:13] + x[13:18] + rng.normal(size=(5,) + shape[::-1]) * 1e-6
    norm = norm_block(x, dq, 1.0)
    net.set_norm(norm)
    xd = torch.tensor(x, dtype=torch.float32, device="cuda")
    dqd = torch.tensor(dq, dtype=torch.float32, device="cuda")
    acts_b, y, dz_b, g = net.grad_trace(xd, dqd)
    assert np.array_equal(net.params(), p0)  # no update
    layers = cnn.unflatten(p0)
    A = [from_channels_last(bits_to_f64(acts_b[l]), CI[l], shape) for l in range(4)]
    # layer 0 input: the standardised inputs (FP32) rounded to bfloat16
    x32 = x.astype(np.float32)
    xs = cnn.standardise(x32, norm).astype(np.float64)
    flips = {"in": handed_on(A[0], xs, np.abs(xs).max(), "inputs")}
    assert not bits_to_f64(acts_b[0])[:, 18:].any()
    for l in range(4):
        W, b = layers[l]
        z = cnn.conv(A[l], cnn.bf16(W), b).numpy()
        if l < 3:
            flips[f"a{l + 1}"] = handed_on(A[l + 1], np.maximum(z, 0.0), np.abs(z).max(), f"act {l + 1}")
        else:
            ey = rel(from_channels_last(y, 5, shape), z)
            say("last layer output rel err (teacher-forced):", ey)
            assert ey <= 1e-5
    # loss gradient: 2 (y - t) / (5 N) with the standardised target in FP32
    c = dq.astype(np.float32) - x32[8:13] - np.float32(1.0) * x32[13:18]
    t = (c - norm[cnn.OUT_MEAN:cnn.OUT_MEAN + 5, None, None, None]) / norm[cnn.OUT_STD:cnn.OUT_STD + 5, None, None, None]
    yg = from_channels_last(y, 5, shape).astype(np.float64)
    dz3 = 2.0 * (yg - t.astype(np.float64)) / yg.size
    DZ = [from_channels_last(bits_to_f64(dz_b[l]), CO[l], shape) for l in range(4)]
    flips["dz3"] = handed_on(DZ[3], dz3, np.abs(dz3).max(), "loss gradient")
    assert not bits_to_f64(dz_b[3])[:, 5:].any()
    starts = np.cumsum([0] + [co * ci * 27 + co for co, ci, *_ in cnn.layer_shapes()])
    for l in range(3, -1, -1):
        W, _ = layers[l]
        dW, db, dx = cnn.layer_backward(A[l], DZ[l], cnn.bf16(W))
        gl = g[starts[l]:starts[l + 1]]
        ew = rel(gl[:-CO[l]], dW.reshape(-1).numpy())
        eb = rel(gl[-CO[l]:], db.numpy())
        say(f"layer {l} teacher-forced grad rel err: dW {ew:.2e} db {eb:.2e}")
        assert ew <= 1e-5 and eb <= 1e-5
        if l > 0:
            dzp = dx.numpy() * (A[l] > 0)
            flips[f"dz{l - 1}"] = handed_on(DZ[l - 1], dzp, np.abs(dzp).max(), f"dz {l - 1}")
    say("entries rounded to the other bfloat16 neighbour (of", A[0].size, "per 18-32 channels):", flips)
    # free-running: the oracle's own activations and gradient.  The two sides
    # round the counted entries to different neighbours; the bar for the
    # output is three times what the same number of one-ulp changes at random
    # entries of the oracle's activations does to its output (at least 1e-3).
    acts_o, z_o = cnn.forward(p0, xs)
    ef = rel(yg, z_o.numpy())
    gref = cnn.backward(p0, acts_o, z_o, t).numpy()
    eg = rel(g, gref)
    effect = flip_effect(p0, acts_o, z_o.numpy(), [flips[f"a{l}"] for l in (1, 2, 3)], rng)
    bar = max(1e-3, 3 * effect)
    say(f"free-running: output rel err {ef:.2e} (bar {bar:.2e}: one-ulp changes at as many entries move it "
        f"by {effect:.2e}), gradient rel err {eg:.2e}")
    assert ef <= bar and eg <= 1e-3


def flip_effect(params, acts, z, counts, rng, trials=4):
    """Largest relative change of the network output, over a few trials,
    when counts[l - 1] random non-zero entries of the oracle's bfloat16
    activation l (l = 1, 2, 3) move to the next bfloat16 value and the layers
    after it are evaluated again with the oracle's rounding."""
    layers = cnn.unflatten(params)
    worst = 0.0
    for _ in range(trials):
        h = None
        for l in range(4):
            a = (acts[l] if h is None else h).clone()
            if l >= 1 and counts[l - 1]:
                flat = a.reshape(-1)
                nz = torch.nonzero(flat).reshape(-1).numpy()
                idx = rng.choice(nz, size=min(counts[l - 1], nz.size), replace=False)
                v = flat[idx]
                up = torch.nextafter(v.to(torch.bfloat16), torch.full_like(v.to(torch.bfloat16), float("inf")))
                flat[idx] = up.to(torch.float64)
            W, b = layers[l]
            zz = cnn.conv(a, cnn.bf16(W), b)
            h = cnn.bf16(torch.relu(zz)) if l < 3 else zz
        worst = max(worst, rel(h.numpy(), z))
    return worst
