"""FP64 CPU oracle of the 3D convolutional surrogate (test infrastructure only).

Network: four 3x3x3 convolutions with periodic padding, channels 18 -> 32 ->
32 -> 32 -> 5, bias, ReLU after the first three.  Input channels: the five
stored Q components, the three velocity components, the last increment of Q
over k solver steps (d1) and the change of that increment (s2), standardised
per channel; output: the standardised correction of the next k-step
increment with respect to the extrapolation d1 + beta s2.

Numerics of the GPU kernels that the oracle reproduces: operands (weights
and input activations of every layer, and upstream gradients in the backward
pass) are rounded to bfloat16 (round to nearest even); products are summed
exactly here (FP64) where the GPU sums them in FP32; bias and ReLU act on the
sum; the ReLU output is rounded to bfloat16 again as the next layer's input.

Plain PyTorch CPU ops in float64: ``conv3d`` on a circularly padded input is
the convolution primitive (cross-correlation, tap (kz, ky, kx) reads the input
at offset (kx-1, ky-1, kz-1)); autograd supplies the backward pass.
Arrays are [c][z][y][x].
"""
from __future__ import annotations

import numpy as np
import torch
import torch.nn.functional as F

CHANNELS = (18, 32, 32, 32, 5)
N_LAYERS = 4


def layer_shapes():
    return [(CHANNELS[i + 1], CHANNELS[i], 3, 3, 3) for i in range(N_LAYERS)]


def param_count():
    return sum(co * ci * 27 + co for co, ci, *_ in layer_shapes())


def unflatten(params):
    """Flat FP32/FP64 vector -> [(W, b)] per layer (PyTorch Conv3d order)."""
    p = torch.as_tensor(np.asarray(params, dtype=np.float64))
    out, k = [], 0
    for co, ci, *_ in layer_shapes():
        nW = co * ci * 27
        W = p[k:k + nW].reshape(co, ci, 3, 3, 3)
        k += nW
        b = p[k:k + co]
        k += co
        out.append((W, b))
    assert k == p.numel()
    return out


def bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    x = torch.as_tensor(x)
    return x.to(torch.float32).to(torch.bfloat16).to(torch.float64)


def conv(x, W, b=None):
    """Periodic 3x3x3 convolution: x [ci, z, y, x] -> [co, z, y, x]."""
    xp = F.pad(torch.as_tensor(x, dtype=torch.float64)[None], (1, 1, 1, 1, 1, 1), mode="circular")
    y = F.conv3d(xp, torch.as_tensor(W, dtype=torch.float64))[0]
    if b is not None:
        y = y + torch.as_tensor(b, dtype=torch.float64)[:, None, None, None]
    return y


def conv_sites(x, W, b, sites):
    """The periodic convolution at selected sites only (direct sums): x [ci,
    z, y, x], sites an array of (z, y, x) rows -> [len(sites), co]."""
    x = np.asarray(x, dtype=np.float64)
    W = np.asarray(W, dtype=np.float64)
    _, nz, ny, nx = x.shape
    out = np.zeros((len(sites), W.shape[0]))
    for n, (z, y, xx) in enumerate(np.asarray(sites)):
        patch = np.empty((x.shape[0], 3, 3, 3))
        for kz in range(3):
            for ky in range(3):
                for kx in range(3):
                    patch[:, kz, ky, kx] = x[:, (z + kz - 1) % nz, (y + ky - 1) % ny, (xx + kx - 1) % nx]
        out[n] = np.tensordot(W, patch, axes=([1, 2, 3, 4], [0, 1, 2, 3]))
        if b is not None:
            out[n] += np.asarray(b, dtype=np.float64)
    return out


def forward(params, x_std, rounding=True):
    """Full network on standardised inputs x_std [18, z, y, x].

    Returns (activations, z_last): activations[l] is the (rounded) input of
    layer l, z_last the FP64 output of the last layer (standardised dQ)."""
    r = bf16 if rounding else (lambda t: torch.as_tensor(t, dtype=torch.float64))
    layers = unflatten(params)
    acts = [r(x_std)]
    h = acts[0]
    for l, (W, b) in enumerate(layers):
        z = conv(h, r(W), b)
        if l < N_LAYERS - 1:
            h = r(torch.relu(z))
            acts.append(h)
        else:
            return acts, z
    raise AssertionError


def layer_backward(x, dz, W):
    """Gradients of one layer given its input x [ci,...], the gradient dz
    [co,...] of the loss with respect to its pre-activation output and its
    weights W: returns (dW, db, dx) in FP64 (dx before any ReLU mask)."""
    xt = torch.as_tensor(x, dtype=torch.float64).clone().requires_grad_(True)
    Wt = torch.as_tensor(W, dtype=torch.float64).clone().requires_grad_(True)
    bt = torch.zeros(Wt.shape[0], dtype=torch.float64, requires_grad=True)
    z = conv(xt, Wt, bt)
    dW, db, dx = torch.autograd.grad(z, (Wt, bt, xt), grad_outputs=torch.as_tensor(dz, dtype=torch.float64))
    return dW, db, dx


def mse(z_last, target):
    """Mean over sites and the five output channels of (z - t)^2."""
    d = torch.as_tensor(z_last, dtype=torch.float64) - torch.as_tensor(target, dtype=torch.float64)
    return float((d * d).mean())


def backward(params, acts, z_last, target, rounding=True):
    """Gradient of the MSE loss for every layer, with the GPU's rounding of
    the upstream gradients (bfloat16) and of the weights.  Returns the flat
    FP64 gradient vector."""
    r = bf16 if rounding else (lambda t: torch.as_tensor(t, dtype=torch.float64))
    layers = unflatten(params)
    n = z_last.numel()
    dz = r(2.0 * (torch.as_tensor(z_last) - torch.as_tensor(target, dtype=torch.float64)) / n)
    grads = [None] * N_LAYERS
    for l in range(N_LAYERS - 1, -1, -1):
        W, _ = layers[l]
        dW, db, dx = layer_backward(acts[l], dz, r(W))
        grads[l] = (dW, db)
        if l > 0:
            dz = r(dx * (acts[l] > 0))
    return torch.cat([torch.cat([dW.reshape(-1), db]) for dW, db in grads])


def adam(params, grad, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba), FP64; returns (params, m, v)."""
    p = np.asarray(params, dtype=np.float64)
    g = np.asarray(grad, dtype=np.float64)
    m = b1 * np.asarray(m, dtype=np.float64) + (1 - b1) * g
    v = b2 * np.asarray(v, dtype=np.float64) + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


# Layout of the standardisation block: input means and stds, target means and
# stds, and beta.
NIN = CHANNELS[0]
IN_MEAN, IN_STD, OUT_MEAN, OUT_STD, BETA = 0, NIN, 2 * NIN, 2 * NIN + 5, 2 * NIN + 10
NORM_SIZE = 2 * NIN + 11


def standardise(x, norm):
    """Raw inputs x [18, ...] -> (x - mean) / std, in FP32 as the GPU does."""
    x = np.asarray(x, dtype=np.float32)
    m = np.asarray(norm[IN_MEAN:IN_MEAN + NIN], dtype=np.float32).reshape((NIN,) + (1,) * (x.ndim - 1))
    s = np.asarray(norm[IN_STD:IN_STD + NIN], dtype=np.float32).reshape((NIN,) + (1,) * (x.ndim - 1))
    return (x - m) / s


def increment(params, norm, Q, u, d1, s2):
    """Increment of Q over the next k steps predicted from the state (Q, u)
    and the history (d1, s2), all [c, z, y, x]: the extrapolation
    d1 + beta s2 plus the de-standardised network output.  FP64."""
    x = np.concatenate([np.asarray(Q, dtype=np.float32), np.asarray(u, dtype=np.float32),
                        np.asarray(d1, dtype=np.float32), np.asarray(s2, dtype=np.float32)])
    _, z = forward(params, standardise(x, norm))
    sd = np.asarray(norm[OUT_STD:OUT_STD + 5], dtype=np.float64)[:, None, None, None]
    mu = np.asarray(norm[OUT_MEAN:OUT_MEAN + 5], dtype=np.float64)[:, None, None, None]
    beta = float(norm[BETA])
    return np.asarray(d1, dtype=np.float64) + beta * np.asarray(s2, dtype=np.float64) + z.numpy() * sd + mu


def jump(params, norm, Q, u, d1, s2):
    """One surrogate jump: Q += dq with the history advanced (s2 = dq - d1,
    d1 = dq).  Returns (Q, d1, s2) in FP64."""
    dq = increment(params, norm, Q, u, d1, s2)
    return np.asarray(Q, dtype=np.float64) + dq, dq, dq - np.asarray(d1, dtype=np.float64)
