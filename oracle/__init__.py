"""FP64 CPU oracle of the hybrid lattice-Boltzmann step (test infrastructure).

Only the test suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It wraps the plain C library built from
``hlb_oracle.c`` (see that file for the equations each routine follows) and
shares no code with the HIP path.

Arrays are numpy float64, structure-of-arrays, component-major
``[c][z][y][x]`` (x fastest).  Q is the full 3x3 tensor, nine planes indexed
``3a+b``; ``q5_to_q9``/``q9_to_q5`` convert from/to the five stored components
(xx, xy, xz, yy, yz).  LB populations are deviations ``g_i = f_i - w_i rho0``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hlb_oracle.c")
_LIB = os.environ.get("HLB_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
          "-std=c11", "-Wall", "-Wextra"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Params(ctypes.Structure):
    """Mirror of ``or_params`` in hlb_oracle.c."""

    _fields_ = [
        ("tau", ctypes.c_double),
        ("rho0", ctypes.c_double),
        ("A0", ctypes.c_double),
        ("gamma", ctypes.c_double),
        ("K", ctypes.c_double),
        ("q0", ctypes.c_double),
        ("Gamma", ctypes.c_double),
        ("xi", ctypes.c_double),
        ("flow", ctypes.c_int),
        ("lb_model", ctypes.c_int),
    ]


def flow_code(flow=True, coupling="force") -> int:
    """0: u == 0; 1: whole stress as a body force; 2: split coupling."""
    if coupling not in ("force", "split"):
        raise ValueError(f"coupling {coupling!r}")
    return 0 if not flow else (2 if coupling == "split" else 1)


LB_MODELS = {"d3q19": 0, "d3q15": 1}


def params(tau=2.5, rho0=1.0, A0=0.01, gamma=3.0, K=0.0, q0=0.0, Gamma=0.3, xi=0.7,
           flow=True, coupling="force", lb_model="d3q19") -> Params:
    """lb_model: "d3q19" (BGK with second-order forcing) or "d3q15" (the
    paper's predictor-corrector scheme)."""
    return Params(tau, rho0, A0, gamma, K, q0, Gamma, xi, flow_code(flow, coupling), LB_MODELS[lb_model])


def n_pop(p: Params) -> int:
    return 15 if p.lb_model == 1 else 19


_lib = None


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        pp = ctypes.POINTER(Params)
        I = ctypes.c_int
        L.or_lattice.argtypes = [ip, dp]
        L.or_q5_to_q9.argtypes = [ctypes.c_long, dp, dp]
        L.or_q9_to_q5.argtypes = [ctypes.c_long, dp, dp]
        L.or_chem.argtypes = [pp, I, I, I, dp, dp, dp, dp]
        L.or_force.argtypes = [pp, I, I, I, dp, dp]
        L.or_rhs.argtypes = [pp, I, I, I, dp, dp, dp]
        L.or_qupdate.argtypes = [pp, I, I, I, dp, dp, dp]
        L.or_lb.argtypes = [pp, I, I, I, dp, dp, dp, dp, dp]
        L.or_split.argtypes = [pp, I, I, I, dp, dp, dp]
        L.or_lb_split.argtypes = [pp, I, I, I, dp, dp, dp, dp, dp, dp]
        L.or_lb_pc.argtypes = [pp, I, I, I, dp, dp, dp, dp, dp, dp]
        L.or_init_g.argtypes = [pp, I, I, I, dp, dp, dp]
        L.or_readout.argtypes = [pp, I, I, I, dp, dp, dp, dp]
        L.or_step.argtypes = [pp, I, I, I, dp, dp, I]
        L.or_sum.argtypes = [dp, ctypes.c_long]
        L.or_sum.restype = ctypes.c_double
        L.or_totals.argtypes = [pp, I, I, I, dp, dp, dp, dp, dp]
        L.or_set_threads.argtypes = [I]
        L.or_max_threads.restype = I
        _lib = L
    return _lib


def set_threads(n):
    """Thread count of the oracle's OpenMP loops (for timing runs)."""
    lib().or_set_threads(int(n))


def max_threads():
    return int(lib().or_max_threads())


def _p(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _shape(a):
    # arrays are [c][z][y][x]; returns (nx, ny, nz)
    return a.shape[-1], a.shape[-2], a.shape[-3]


def lattice():
    e = np.zeros((19, 3), dtype=np.int32)
    w = np.zeros(19)
    lib().or_lattice(e.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _p(w))
    return e, w


def q5_to_q9(Q5):
    Q5 = np.ascontiguousarray(Q5, dtype=np.float64)
    out = np.empty((9,) + Q5.shape[1:])
    lib().or_q5_to_q9(Q5[0].size, _p(Q5), _p(out))
    return out


def q9_to_q5(Q9):
    Q9 = np.ascontiguousarray(Q9, dtype=np.float64)
    out = np.empty((5,) + Q9.shape[1:])
    lib().or_q9_to_q5(Q9[0].size, _p(Q9), _p(out))
    return out


def chem(p: Params, Q9):
    """Molecular field H (9 planes), free-energy density f, stress Pi (9)."""
    Q9 = np.ascontiguousarray(Q9, dtype=np.float64)
    nx, ny, nz = _shape(Q9)
    H = np.empty_like(Q9)
    f = np.empty(Q9.shape[1:])
    Pi = np.empty_like(Q9)
    lib().or_chem(ctypes.byref(p), nx, ny, nz, _p(Q9), _p(H), _p(f), _p(Pi))
    return H, f, Pi


def force(p: Params, Q9):
    Q9 = np.ascontiguousarray(Q9, dtype=np.float64)
    nx, ny, nz = _shape(Q9)
    F = np.empty((3,) + Q9.shape[1:])
    lib().or_force(ctypes.byref(p), nx, ny, nz, _p(Q9), _p(F))
    return F


def split(p: Params, Q9):
    """Split coupling: (sigma^xi (9 planes), body force b (3))."""
    Q9 = np.ascontiguousarray(Q9, dtype=np.float64)
    nx, ny, nz = _shape(Q9)
    sig = np.empty_like(Q9)
    b = np.empty((3,) + Q9.shape[1:])
    lib().or_split(ctypes.byref(p), nx, ny, nz, _p(Q9), _p(sig), _p(b))
    return sig, b


def rhs(p: Params, Q9, u3):
    Q9 = np.ascontiguousarray(Q9, dtype=np.float64)
    u3 = np.ascontiguousarray(u3, dtype=np.float64)
    nx, ny, nz = _shape(Q9)
    R = np.empty_like(Q9)
    lib().or_rhs(ctypes.byref(p), nx, ny, nz, _p(Q9), _p(u3), _p(R))
    return R


def qupdate(p: Params, Q9, u3):
    Q9 = np.ascontiguousarray(Q9, dtype=np.float64)
    u3 = np.ascontiguousarray(u3, dtype=np.float64)
    nx, ny, nz = _shape(Q9)
    out = np.empty_like(Q9)
    lib().or_qupdate(ctypes.byref(p), nx, ny, nz, _p(Q9), _p(u3), _p(out))
    return out


def lb(p: Params, g, F3=None):
    """One pull/collide/force LB step; returns (g_new, rho, u)."""
    g = np.ascontiguousarray(g, dtype=np.float64)
    nx, ny, nz = _shape(g)
    if F3 is not None:
        F3 = np.ascontiguousarray(F3, dtype=np.float64)
    gn = np.empty_like(g)
    rho = np.empty(g.shape[1:])
    u = np.empty((3,) + g.shape[1:])
    lib().or_lb(ctypes.byref(p), nx, ny, nz, _p(g), _p(F3), _p(gn), _p(rho), _p(u))
    return gn, rho, u


def lb_split(p: Params, g, b3, sig9):
    """LB step of the split coupling (body force b3, equilibrium stress sig9)."""
    g = np.ascontiguousarray(g, dtype=np.float64)
    b3 = np.ascontiguousarray(b3, dtype=np.float64)
    sig9 = np.ascontiguousarray(sig9, dtype=np.float64)
    nx, ny, nz = _shape(g)
    gn = np.empty_like(g)
    rho = np.empty(g.shape[1:])
    u = np.empty((3,) + g.shape[1:])
    lib().or_lb_split(ctypes.byref(p), nx, ny, nz, _p(g), _p(b3), _p(sig9), _p(gn), _p(rho), _p(u))
    return gn, rho, u


def lb_pc(p: Params, g, b3=None, sig9=None):
    """One step of the paper's D3Q15 predictor-corrector LB with body force b3
    and equilibrium stress sig9 (either may be None); returns (g_new, rho, u)
    with rho, u the moments of the input populations."""
    g = np.ascontiguousarray(g, dtype=np.float64)
    assert g.shape[0] == 15
    nx, ny, nz = _shape(g)
    if b3 is not None:
        b3 = np.ascontiguousarray(b3, dtype=np.float64)
    if sig9 is not None:
        sig9 = np.ascontiguousarray(sig9, dtype=np.float64)
    gn = np.empty_like(g)
    rho = np.empty(g.shape[1:])
    u = np.empty((3,) + g.shape[1:])
    lib().or_lb_pc(ctypes.byref(p), nx, ny, nz, _p(g), _p(b3), _p(sig9), _p(gn), _p(rho), _p(u))
    return gn, rho, u


def init_g(p: Params, rho, u3):
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    u3 = np.ascontiguousarray(u3, dtype=np.float64)
    nx, ny, nz = _shape(u3)
    g = np.empty((n_pop(p),) + rho.shape)
    lib().or_init_g(ctypes.byref(p), nx, ny, nz, _p(rho), _p(u3), _p(g))
    return g


def readout(p: Params, g, Q9):
    g = np.ascontiguousarray(g, dtype=np.float64)
    Q9 = np.ascontiguousarray(Q9, dtype=np.float64)
    nx, ny, nz = _shape(Q9)
    rho = np.empty(Q9.shape[1:])
    u = np.empty((3,) + Q9.shape[1:])
    lib().or_readout(ctypes.byref(p), nx, ny, nz, _p(g), _p(Q9), _p(rho), _p(u))
    return rho, u


def totals(p: Params, g, Q9):
    g = np.ascontiguousarray(g, dtype=np.float64)
    Q9 = np.ascontiguousarray(Q9, dtype=np.float64)
    nx, ny, nz = _shape(Q9)
    mass = ctypes.c_double()
    mom = np.zeros(3)
    ftot = ctypes.c_double()
    lib().or_totals(ctypes.byref(p), nx, ny, nz, _p(g), _p(Q9), ctypes.byref(mass), _p(mom),
                    ctypes.byref(ftot))
    return mass.value, mom, ftot.value


def psum(v):
    v = np.ascontiguousarray(v, dtype=np.float64).ravel()
    return lib().or_sum(_p(v), v.size)


class State:
    """Oracle state (g, Q9) advanced in place by :meth:`step`."""

    def __init__(self, p: Params, Q5, u3=None, rho=None):
        Q5 = np.ascontiguousarray(Q5, dtype=np.float64)
        shape = Q5.shape[1:]
        if u3 is None:
            u3 = np.zeros((3,) + shape)
        if rho is None:
            rho = np.full(shape, p.rho0)
        self.p = p
        self.Q9 = q5_to_q9(Q5)
        self.g = init_g(p, rho, u3)

    @property
    def shape(self):
        return _shape(self.Q9)

    def step(self, n=1):
        nx, ny, nz = self.shape
        lib().or_step(ctypes.byref(self.p), nx, ny, nz, _p(self.g), _p(self.Q9), int(n))

    def fields(self):
        """(Q5, u, rho) at the current time level."""
        rho, u = readout(self.p, self.g, self.Q9)
        return q9_to_q5(self.Q9), u, rho

    def totals(self):
        return totals(self.p, self.g, self.Q9)
