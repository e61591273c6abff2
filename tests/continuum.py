"""Continuum (spectral, autograd) evaluation of the Beris-Edwards quantities.

Test-only helper that derives, independently of the oracle's hand-written
formulas, the molecular field and the body force of a smooth periodic field:

* H is obtained from the printed free-energy density (Sec. 2.1, Eq. (1) plus
  the divergence term of the one-constant approximation) by the Euler-Lagrange
  equation, with df/dQ and df/d(grad Q) taken by torch autograd and the outer
  divergence taken spectrally; then H = -[sym(G) - tr(G)/3 I] (Eq. (2)).
* The gradient part of the force comes from the identity of Sec. 2.2, Eq. (21):
  d_b(f d_ab - d_a Q_gn df/dQ_gn,b) = -H_gn d_a Q_gn,
  so the oracle's explicit stress gradient term is checked against it.

Fields live on a box of side 2 pi sampled at L points per axis (spacing
h = 2 pi / L); arrays are [c][z][y][x].
"""
from __future__ import annotations

import math

import numpy as np
import torch

EPS = np.zeros((3, 3, 3))
for a, b, c in [(0, 1, 2), (1, 2, 0), (2, 0, 1)]:
    EPS[a, b, c] = 1.0
    EPS[a, c, b] = -1.0


def spectral_d(field, axis_xyz):
    """d/dx_axis of a periodic field sampled on [0, 2 pi)^3 (last three axes z,y,x)."""
    L = field.shape[-1 - axis_xyz]
    ax = field.ndim - 1 - axis_xyz
    F = np.fft.fft(field, axis=ax)
    k = np.fft.fftfreq(L, d=1.0 / L)
    if L % 2 == 0:
        k[L // 2] = 0.0
    shape = [1] * field.ndim
    shape[ax] = L
    return np.real(np.fft.ifft(F * (1j * k).reshape(shape), axis=ax))


def q5_to_full(Q5):
    xx, xy, xz, yy, yz = Q5
    zz = -xx - yy
    return np.stack([np.stack([xx, xy, xz]), np.stack([xy, yy, yz]), np.stack([xz, yz, zz])])


def free_energy_torch(q, p, A0, gamma, K, q0):
    """f of Eq. (1) + K/2 (d_b Q_ab)^2; q: [3,3,P], p: [3(g),3,3,P] = d_g Q_ab."""
    eps = torch.tensor(EPS, dtype=q.dtype)
    qq = torch.einsum("abP,abP->P", q, q)
    q3 = torch.einsum("abP,bcP,caP->P", q, q, q)
    bulk = 0.5 * A0 * (1 - gamma / 3) * qq - A0 * gamma / 3 * q3 + 0.25 * A0 * gamma * qq * qq
    div = torch.einsum("babP->aP", p)
    M = torch.einsum("agd,gdbP->abP", eps, p) + 2 * q0 * q
    return bulk + 0.5 * K * (div * div).sum(0) + 0.5 * K * (M * M).sum((0, 1))


def field_derivs(Q):
    """dQ[g] = d_g Q for a full [3,3,...] periodic field."""
    return np.stack([spectral_d(Q, g) for g in range(3)])


def molecular_field(Q5, A0, gamma, K, q0):
    """Continuum H (full 3x3 per point) by Euler-Lagrange from the free energy."""
    Q = q5_to_full(Q5)
    dQ = field_derivs(Q)
    shp = Q.shape[2:]
    P = int(np.prod(shp))
    q = torch.tensor(Q.reshape(3, 3, P), requires_grad=True)
    p = torch.tensor(dQ.reshape(3, 3, 3, P), requires_grad=True)
    f = free_energy_torch(q, p, A0, gamma, K, q0).sum()
    dfdq, dfdp = torch.autograd.grad(f, (q, p))
    dfdq = dfdq.numpy().reshape(3, 3, *shp)
    dfdp = dfdp.numpy().reshape(3, 3, 3, *shp)
    G = dfdq - sum(spectral_d(dfdp[g], g) for g in range(3))
    sym = 0.5 * (G + np.swapaxes(G, 0, 1))
    tr = G[0, 0] + G[1, 1] + G[2, 2]
    H = -sym
    for a in range(3):
        H[a, a] += tr / 3.0
    return Q, dQ, H


def free_energy_density(Q5, A0, gamma, K, q0):
    Q = q5_to_full(Q5)
    dQ = field_derivs(Q)
    shp = Q.shape[2:]
    P = int(np.prod(shp))
    with torch.no_grad():
        f = free_energy_torch(torch.tensor(Q.reshape(3, 3, P)), torch.tensor(dQ.reshape(3, 3, 3, P)),
                              A0, gamma, K, q0)
    return f.numpy().reshape(shp)


def body_force(Q5, A0, gamma, K, q0, xi):
    """Continuum b_a = -H:d_a Q + d_b (sigma^xi + tau)_ab (Eqs. (7), (8), (21))."""
    Q, dQ, H = molecular_field(Q5, A0, gamma, K, q0)
    I = np.eye(3).reshape(3, 3, *([1] * (Q.ndim - 2)))
    A = Q + I / 3.0
    mm = lambda X, Y: np.einsum("ac...,cb...->ab...", X, Y)
    QH = np.einsum("ab...,ab...->...", Q, H)
    sig = 2 * xi * A * QH - xi * mm(H, A) - xi * mm(A, H)
    tau = mm(Q, H) - mm(H, Q)
    T = sig + tau
    F = np.zeros((3,) + Q.shape[2:])
    for a in range(3):
        F[a] = -np.einsum("gn...,gn...->...", H, dQ[a])
        for b in range(3):
            F[a] += spectral_d(T[a, b], b)
    return F


def split_terms(Q5, A0, gamma, K, q0, xi):
    """Continuum split coupling (Eqs. (17)-(21)): the symmetric xi-stress
    sigma^xi (full 3x3 per point) and the body force
    b_a = d_b tau_ab - H:d_a Q."""
    Q, dQ, H = molecular_field(Q5, A0, gamma, K, q0)
    I = np.eye(3).reshape(3, 3, *([1] * (Q.ndim - 2)))
    A = Q + I / 3.0
    mm = lambda X, Y: np.einsum("ac...,cb...->ab...", X, Y)
    QH = np.einsum("ab...,ab...->...", Q, H)
    sig = 2 * xi * A * QH - xi * mm(H, A) - xi * mm(A, H)
    tau = mm(Q, H) - mm(H, Q)
    b = np.zeros((3,) + Q.shape[2:])
    for a in range(3):
        b[a] = -np.einsum("gn...,gn...->...", H, dQ[a])
        for c in range(3):
            b[a] += spectral_d(tau[a, c], c)
    return sig, b
