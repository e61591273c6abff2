"""FP64 CPU oracle of the polarised-light texture (test infrastructure only;
shares no code with the HIP path).

Sec. 2.3: the sample is a stack of layers of thickness h along the beam (z);
the layer at site r acts on the Stokes vector through the Mueller matrix of
a linear retarder whose axis makes the angle beta(r) with x in the (x, y)
plane and whose retardance is
    delta = 2 pi q h / lambda * (n_o n_e / sqrt(n_o^2 sin^2 alpha + n_e^2 cos^2 alpha) - n_o),
alpha the angle between the director and the beam (cos alpha = d_z), q the
local order (largest eigenvalue of Q), d the director.  Polariser and
analyser are linear polarisers at angles phi_in and phi_out to x; the image is
the first Stokes component S0 behind the analyser, summed over wavelengths
with weights.  Light enters at z = 0: the layer z = 0 acts first.

Readings (where the printed formulas and the text disagree):
  * beta = atan2(d_y, d_x), the angle of the director's projection to the x
    axis, as the text states and as the printed retarder matrix requires;
  * the polariser matrix takes the Stokes angle 2 phi (cos 2 phi, sin 2 phi),
    so that phi_in = 0, phi_out = pi/2 is the crossed pair the text names;
  * unpolarised input light S_in = (1, 0, 0, 0).

q and d come from ``oracle.order`` (numpy eigh per site).  Arrays are
[c][z][y][x]; the image is [y][x].
"""
from __future__ import annotations

import numpy as np

from . import order as _order

N_O, N_E = 1.5, 2.0
WAVELENGTHS = (16.0, 18.0, 20.0)
WEIGHTS = (0.2, 0.6, 0.2)


def layer_angles(q, d, lam, h=1.0, n_o=N_O, n_e=N_E):
    """(cos 2 beta, sin 2 beta, delta) per site."""
    dx, dy, dz = d
    cos_a = np.clip(dz, -1.0, 1.0)
    sin2_a = 1.0 - cos_a ** 2
    beta = np.arctan2(dy, dx)
    neff = n_o * n_e / np.sqrt(n_o ** 2 * sin2_a + n_e ** 2 * cos_a ** 2)
    delta = 2 * np.pi * q * h / lam * (neff - n_o)
    return np.cos(2 * beta), np.sin(2 * beta), delta


def retarder(cb, sb, delta):
    """Mueller matrix of each layer as printed, [4][4][...]."""
    cd, sd = np.cos(delta), np.sin(delta)
    z, o = np.zeros_like(cb), np.ones_like(cb)
    return np.array([
        [o, z, z, z],
        [z, cb ** 2 + sb ** 2 * cd, cb * sb * (1 - cd), -sb * sd],
        [z, cb * sb * (1 - cd), sb ** 2 + cb ** 2 * cd, cb * sd],
        [z, sb * sd, -cb * sd, cd],
    ])


def polariser(phi):
    c, s = np.cos(2 * phi), np.sin(2 * phi)
    return 0.5 * np.array([[1, c, s, 0], [c, c * c, c * s, 0], [s, s * c, s * s, 0], [0, 0, 0, 0]])


def stokes_out(q, d, lam, phi_in=0.0, phi_out=np.pi / 2, h=1.0, n_o=N_O, n_e=N_E, s_in=(1.0, 0.0, 0.0, 0.0)):
    """Stokes vector behind the analyser, [4][y][x], for one wavelength."""
    cb, sb, delta = layer_angles(q, d, lam, h, n_o, n_e)
    nz, ny, nx = q.shape
    S = np.einsum("ab,b->a", polariser(phi_in), np.asarray(s_in, dtype=np.float64))
    S = np.broadcast_to(S[:, None, None], (4, ny, nx)).copy()
    for z in range(nz):  # the beam meets layer z = 0 first
        M = retarder(cb[z], sb[z], delta[z])
        S = np.einsum("abyx,byx->ayx", M, S)
    return np.einsum("ab,byx->ayx", polariser(phi_out), S)


def image(Q5, wavelengths=WAVELENGTHS, weights=WEIGHTS, phi_in=0.0, phi_out=np.pi / 2, h=1.0, n_o=N_O,
          n_e=N_E):
    """Weighted S0 behind the analyser, [y][x]."""
    q, d, _, _ = _order.order(Q5)
    out = 0.0
    for lam, w in zip(wavelengths, weights):
        out = out + w * stokes_out(q, d, lam, phi_in, phi_out, h, n_o, n_e)[0]
    return out
