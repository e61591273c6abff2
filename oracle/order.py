"""FP64 CPU oracle of the local order and disclination analysis (test
infrastructure only; shares no code with the HIP path).

Sec. 2.1: the local magnitude of order q(r) is the largest eigenvalue of Q,
and a lattice site belongs to a disclination when q falls below a threshold
(0.19 in the paper's runs).  Sec. 2.3: the director d(r) is the normalised
eigenvector of that largest eigenvalue.  The eigen-decomposition is the
library's symmetric solver (numpy ``eigh``, LAPACK) on the full 3x3 tensor
of every site, in float64.

Arrays are [c][z][y][x]; Q5 holds the stored components (xx, xy, xz, yy, yz)
with Q_zz = -Q_xx - Q_yy.
"""
from __future__ import annotations

import numpy as np

THRESHOLD = 0.19


def full_tensor(Q5):
    """[..., 3, 3] per site from the five stored components ([5][z][y][x])."""
    xx, xy, xz, yy, yz = (np.asarray(Q5[k], dtype=np.float64) for k in range(5))
    zz = -xx - yy
    rows = [np.stack([xx, xy, xz], -1), np.stack([xy, yy, yz], -1), np.stack([xz, yz, zz], -1)]
    return np.stack(rows, -2)


def order(Q5, threshold=THRESHOLD):
    """(q, d, defect, gap): largest eigenvalue q [z][y][x], its unit eigenvector
    d [3][z][y][x] (sign as the solver returns it), defect = q < threshold,
    and gap = q minus the middle eigenvalue (how well d is determined)."""
    Q = full_tensor(Q5)
    w, v = np.linalg.eigh(Q)  # ascending eigenvalues, eigenvectors in columns
    q = w[..., 2]
    d = np.moveaxis(v[..., :, 2], -1, 0)
    return q, d, q < threshold, w[..., 2] - w[..., 1]


def defects_per_plane(defect):
    """Number of disclination sites in each z-plane."""
    return np.asarray(defect, dtype=np.int64).sum(axis=(1, 2))
