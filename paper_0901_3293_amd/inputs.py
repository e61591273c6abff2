"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module holds initial states and parameter sets only -- none of the
method's arithmetic.  Both the HIP path and the CPU oracle receive the very
same arrays from here.

Layout: numpy float64, component-major ``[c][z][y][x]`` (x fastest); Q as the
five stored components (xx, xy, xz, yy, yz) with Q_zz = -Q_xx - Q_yy.

Parameter definitions (Sec. 2.1, Eqs. (9)-(10)): chirality
``kappa = sqrt(108 K q0^2 / (A0 gamma))`` and reduced temperature
``tau = 27 (1 - gamma/3) / gamma``; the one elastic constant K plays the role
of L1 there.  A0 = 0.01 throughout; Gamma = 0.3 and xi = 0.7 are the kinetic
values chosen in Sec. 2.1; the LB relaxation time is 2.5.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, asdict

import numpy as np

A0_DEFAULT = 0.01


@dataclass
class PhysParams:
    """Physical parameters of one run (lattice units)."""

    tau: float = 2.5        # LB relaxation time
    rho0: float = 1.0       # reference density
    A0: float = A0_DEFAULT
    gamma: float = 3.0
    K: float = 0.0
    q0: float = 0.0
    Gamma: float = 0.3
    xi: float = 0.7
    flow: bool = True
    coupling: str = "force"  # "force": whole stress as a body force; "split": Sec. 2.2 split
    lb_model: str = "d3q19"  # "d3q19": BGK + second-order forcing; "d3q15": the paper's predictor-corrector

    def as_dict(self):
        return asdict(self)


def gamma_from_tau(tau_ldg: float) -> float:
    """Invert tau = 27 (1 - gamma/3) / gamma (Sec. 2.1, Eq. (10))."""
    return 27.0 / (tau_ldg + 9.0)


def K_from_kappa(kappa: float, gamma: float, q0: float, A0: float = A0_DEFAULT) -> float:
    """Invert kappa = sqrt(108 K q0^2 / (A0 gamma)) (Sec. 2.1, Eq. (9))."""
    return kappa * kappa * A0 * gamma / (108.0 * q0 * q0)


def reduced(kappa: float, tau_ldg: float, q0: float, A0: float = A0_DEFAULT, **kw) -> PhysParams:
    g = gamma_from_tau(tau_ldg)
    return PhysParams(A0=A0, gamma=g, K=K_from_kappa(kappa, g, q0, A0), q0=q0, **kw)


def uniaxial_amplitude(gamma: float) -> float:
    """Scalar order S of the uniaxial bulk minimum of the Landau-de Gennes
    potential of Eq. (1) for Q = S (n n - I/3):  S = 1/4 + 3/4 sqrt(1 - 8/(3 gamma))."""
    return 0.25 + 0.75 * math.sqrt(max(0.0, 1.0 - 8.0 / (3.0 * gamma)))


def _grid(shape):
    nx, ny, nz = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return x.astype(np.float64), y.astype(np.float64), z.astype(np.float64)


def _q5_from_director(n, S):
    nx_, ny_, nz_ = n
    return np.stack([
        S * (nx_ * nx_ - 1.0 / 3.0),
        S * nx_ * ny_,
        S * nx_ * nz_,
        S * (ny_ * ny_ - 1.0 / 3.0),
        S * ny_ * nz_,
    ])


def helix_q5(shape, q0, S, axis="z", phase=0.0):
    """Uniaxial cholesteric helix Q = S (n n - I/3).

    axis z: n = (cos t, sin t, 0), t = q0 z + phase; x and y follow by cyclic
    permutation: axis x: n = (0, cos t, sin t); axis y: n = (sin t, 0, cos t).
    """
    x, y, z = _grid(shape)
    zero = np.zeros_like(x)
    if axis == "z":
        t = q0 * z + phase
        n = (np.cos(t), np.sin(t), zero)
    elif axis == "x":
        t = q0 * x + phase
        n = (zero, np.cos(t), np.sin(t))
    elif axis == "y":
        t = q0 * y + phase
        n = (np.sin(t), zero, np.cos(t))
    else:
        raise ValueError(axis)
    return _q5_from_director(n, S)


def o2_q5(shape, q0, A):
    """Double-twist superposition of three orthogonal helices with simple-cubic
    symmetry (the high-chirality O2 structure used as the blue-phase seed).
    Each term is 2A times a helix along one axis, so the period is pi/q0."""
    x, y, z = _grid(shape)
    c = lambda v: np.cos(2.0 * q0 * v)
    s = lambda v: np.sin(2.0 * q0 * v)
    return np.stack([
        A * (c(z) - c(y)),   # xx
        A * s(z),            # xy
        A * s(y),            # xz
        A * (c(x) - c(z)),   # yy
        A * s(x),            # yz
    ])


def noise(shape, amp, seed, ncomp=5):
    """i.i.d. U(-amp, amp) on each stored component (numpy PCG64)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nx, ny, nz = shape
    return rng.uniform(-amp, amp, size=(ncomp, nz, ny, nx))


def rest_fluid(shape, rho0=1.0):
    nx, ny, nz = shape
    return np.zeros((3, nz, ny, nx)), np.full((nz, ny, nx), rho0)


# --------------------------------------------------------------------------
# Workloads
# --------------------------------------------------------------------------

def helix_case(n=32, q0=2.0 * math.pi / 16.0, kappa=1.0, tau_ldg=0.0, noise_amp=1e-4, seed=1,
               flow=True):
    """Cholesteric helix along z with pitch 2 pi/q0 and uniform noise, fluid at
    rest: the 32^3 FP64 parity workload (kappa = 1, tau = 0 as in Sec. 3)."""
    shape = (n, n, n)
    p = reduced(kappa, tau_ldg, q0, flow=flow)
    S = uniaxial_amplitude(p.gamma)
    Q = helix_q5(shape, q0, S, "z") + noise(shape, noise_amp, seed)
    u, rho = rest_fluid(shape, p.rho0)
    return p, Q, u, rho


# Amplitude of the O2 seed that minimises the oracle's total free energy at
# kappa = 0.7, tau = -0.5, q0 = pi/32 (written by tests/golden/make_o2_amplitude.py).
O2_AMPLITUDE_K07_TM05 = None


def o2_amplitude():
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "tests",
                        "golden", "o2_amplitude.json")
    with open(path) as fh:
        return float(json.load(fh)["A"])


def bpii_case(n=128, cell=32, kappa=0.7, tau_ldg=-0.5, A=None, flow=True):
    """Simple-cubic double-twist lattice of (n/cell)^3 unit cells of side `cell`
    (q0 = pi/cell), fluid at rest: the 128^3 throughput workload."""
    if n % cell:
        raise ValueError("lattice must hold whole unit cells")
    q0 = math.pi / cell
    shape = (n, n, n)
    p = reduced(kappa, tau_ldg, q0, flow=flow)
    if A is None:
        A = o2_amplitude()
    Q = o2_q5(shape, q0, A)
    u, rho = rest_fluid(shape, p.rho0)
    return p, Q, u, rho


def slab_case(nx=64, ny=64, nz=256, cell=32, seed_depth=32, kappa=0.8, tau_ldg=0.0, A=None,
              flow=True):
    """Domain-growth slab: O2 seed for z < seed_depth inside a cholesteric helix
    with axis along x (one pitch in nx when q0 = pi/cell and nx = 2 cell)."""
    q0 = math.pi / cell
    shape = (nx, ny, nz)
    p = reduced(kappa, tau_ldg, q0, flow=flow)
    if A is None:
        A = o2_amplitude()
    S = uniaxial_amplitude(p.gamma)
    Q = helix_q5(shape, q0, S, "x")
    seed = o2_q5(shape, q0, A)
    Q[:, :seed_depth] = seed[:, :seed_depth]
    u, rho = rest_fluid(shape, p.rho0)
    return p, Q, u, rho


def replica_set(n_replicas=96, sizes=(24, 32, 48, 64), seed=4, noise_amp=1e-4):
    """Uneven periodic boxes for the batched form: cube side drawn from `sizes`,
    kappa ~ U[0.3, 1.2], tau ~ U[-1, 0.5], a helix along a random axis with a
    random phase (q0 = 2 pi / L, one pitch per box), amplitude S*(gamma), noise."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for r in range(n_replicas):
        L = int(rng.choice(sizes))
        kappa = float(rng.uniform(0.3, 1.2))
        tau_ldg = float(rng.uniform(-1.0, 0.5))
        axis = "xyz"[int(rng.integers(3))]
        phase = float(rng.uniform(0.0, 2.0 * math.pi))
        q0 = 2.0 * math.pi / L
        p = reduced(kappa, tau_ldg, q0)
        shape = (L, L, L)
        Q = helix_q5(shape, q0, uniaxial_amplitude(p.gamma), axis, phase)
        Q += noise(shape, noise_amp, seed * 1000 + r)
        u, rho = rest_fluid(shape, p.rho0)
        out.append(dict(L=L, kappa=kappa, tau_ldg=tau_ldg, params=p, Q=Q, u=u, rho=rho))
    return out


def batch_parity_set():
    """A small uneven set for checking batched runs box by box: seven cubes
    of side 8 to 20 from replica_set (seed 9), the third with the flow off,
    and a non-cubic 10 x 6 x 14 box with a z-helix plus noise 1e-3."""
    rs = replica_set(n_replicas=7, sizes=(8, 12, 16, 20), seed=9)
    rs[2]["params"].flow = False
    Qn = helix_q5((10, 6, 14), 2 * math.pi / 14, 0.4, "z") + noise((10, 6, 14), 1e-3, 5)
    rs.append(dict(L=None, params=reduced(0.8, -0.2, 2 * math.pi / 14), Q=Qn, u=None, rho=None))
    return rs


def smooth_field(shape, amp=0.1, seed=7, modes=2):
    """Smooth periodic symmetric-traceless field: a few random low Fourier modes
    per stored component (for continuum-limit checks)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x, y, z = _grid(shape)
    nx, ny, nz = shape
    comps = []
    for c in range(5):
        v = np.zeros_like(x)
        for _ in range(modes):
            m = rng.integers(-2, 3, size=3)
            ph = rng.uniform(0, 2 * math.pi)
            a = rng.uniform(0.5, 1.0)
            v += a * np.cos(2 * math.pi * (m[0] * x / nx + m[1] * y / ny + m[2] * z / nz) + ph)
        comps.append(amp * v / modes)
    return np.stack(comps)


# --------------------------------------------------------------------------
# Surrogate network
# --------------------------------------------------------------------------

CNN_CHANNELS = (18, 32, 32, 32, 5)


def cnn_params(seed=0, scale=1.0):
    """Seeded He-style initial weights of the 3x3x3 convolutional surrogate as
    one flat FP32 vector, layer by layer: W [co][ci][kz][ky][kx] drawn from
    N(0, scale^2 * 2 / (27 ci)), then a zero bias [co]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for ci, co in zip(CNN_CHANNELS[:-1], CNN_CHANNELS[1:]):
        std = scale * math.sqrt(2.0 / (ci * 27))
        parts.append(rng.normal(0.0, std, size=co * ci * 27))
        parts.append(np.zeros(co))
    return np.concatenate(parts).astype(np.float32)
