"""C-ABI surface checks that need no GPU: the library loads, exports every
function include/hlb.h declares, and its host-only logic (sizes, parameter
mapping and validation, call-order errors, sticky errors) behaves as
documented.  No call here launches device work."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

from paper_0901_3293_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def H():
    from paper_0901_3293_amd import hlb

    return hlb


def declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(hlb\w*)\s*\(", txt))
    return names


def test_exports_every_declared_symbol(H):
    L = H.lib()
    names = declared_functions()
    assert len(names) >= 13
    for n in sorted(names):
        assert hasattr(L, n), n


def test_workspace_bytes(H):
    assert H.workspace_bytes(3, 8, 8) == 0
    assert H.workspace_bytes(8, 8, 8, 7) == 0
    a = H.workspace_bytes(32, 32, 32, H.HLB_FP64)
    b = H.workspace_bytes(32, 32, 32, H.HLB_FP32)
    N = 32 ** 3
    # 19+19 populations, 5+5 Q, u 3, stress or split terms 12, D3Q15 predictor
    # populations 15: 78 values per site plus partials
    assert 78 * 8 * N <= a < 78 * 8 * N + 2 ** 20
    assert 78 * 4 * N <= b < 78 * 4 * N + 2 ** 20


def test_workspace_size_limits(H):
    """Kernels address one field plane with 32-bit byte offsets and index
    sites in 31 bits: FP64 lattices stop below 2^29 sites (a plane of 4 GiB),
    FP32 ones below 2^30."""
    assert H.workspace_bytes(1024, 1024, 511, H.HLB_FP64) > 0
    assert H.workspace_bytes(1024, 1024, 512, H.HLB_FP64) == 0
    assert H.workspace_bytes(1024, 1024, 512, H.HLB_FP32) > 0
    assert H.workspace_bytes(1024, 1024, 1023, H.HLB_FP32) > 0
    assert H.workspace_bytes(1024, 1024, 1024, H.HLB_FP32) == 0
    L = H.lib()
    dims = (ctypes.c_int * 3)(1024, 1024, 512)
    assert L.hlb_batch_workspace_bytes(1, dims, H.HLB_FP64) == 0
    assert L.hlb_batch_workspace_bytes(1, dims, H.HLB_FP32) > 0


def test_fe_from_reduced(H):
    q0 = 2 * math.pi / 16
    fe = H.fe_from_reduced(1.0, 0.0, q0, 0.01)
    assert fe.gamma == pytest.approx(3.0, rel=1e-15)
    # kappa^2 = 108 K q0^2 / (A0 gamma), tau = 27 (1 - gamma/3)/gamma (Sec. 2.1)
    assert math.sqrt(108 * fe.K * q0 ** 2 / (fe.A0 * fe.gamma)) == pytest.approx(1.0, rel=1e-14)
    fe2 = H.fe_from_reduced(0.7, -0.5, math.pi / 32, 0.01)
    assert 27 * (1 - fe2.gamma / 3) / fe2.gamma == pytest.approx(-0.5, rel=1e-14)
    assert fe2.K == pytest.approx(1.49526e-2, rel=1e-5)
    with pytest.raises(H.HlbError):
        H.fe_from_reduced(1.0, 0.0, 0.0, 0.01)


class FakeCtx:
    """A context over a fake (never dereferenced) workspace address: only the
    host-side validation paths are exercised."""

    def __init__(self, H, shape=(8, 8, 8)):
        self.H = H
        L = H.lib()
        self.n = L.hlb_workspace_bytes(*shape, 0)
        self.ctx = ctypes.c_void_p()
        self.rc = L.hlb_create(*shape, 0, ctypes.c_void_p(1 << 40), self.n, None, ctypes.byref(self.ctx))

    def params(self, **kw):
        p = I.PhysParams(K=0.01, q0=0.3)
        for k, v in kw.items():
            setattr(p, k, v)
        H = self.H
        lb = H.LbParams(p.tau, p.rho0)
        fe = H.FeParams(p.A0, p.gamma, p.K, p.q0)
        be = H.BeParams(p.Gamma, p.xi, 1)
        return H.lib().hlb_set_params(self.ctx, ctypes.byref(lb), ctypes.byref(fe), ctypes.byref(be))

    def close(self):
        self.H.lib().hlb_destroy(self.ctx)


def test_create_rejects_bad_arguments(H):
    L = H.lib()
    ctx = ctypes.c_void_p()
    n = L.hlb_workspace_bytes(8, 8, 8, 0)
    assert L.hlb_create(8, 8, 8, 0, None, n, None, ctypes.byref(ctx)) == -1
    assert L.hlb_create(8, 8, 8, 0, ctypes.c_void_p((1 << 40) + 8), n, None, ctypes.byref(ctx)) == -1
    assert L.hlb_create(8, 8, 8, 0, ctypes.c_void_p(1 << 40), n - 1, None, ctypes.byref(ctx)) == -6
    assert L.hlb_create(2, 8, 8, 0, ctypes.c_void_p(1 << 40), n, None, ctypes.byref(ctx)) == -1


@pytest.mark.parametrize("bad", [dict(tau=0.5), dict(rho0=0.0), dict(A0=-1.0), dict(gamma=0.0),
                                 dict(K=-1e-3), dict(Gamma=0.0), dict(K=1.0, Gamma=0.2)])
def test_set_params_validation_is_sticky(H, bad):
    c = FakeCtx(H)
    assert c.rc == 0
    assert c.params(**bad) == -2
    msg = H.lib().hlb_last_error(c.ctx).decode()
    assert msg
    # sticky: a valid call now reports the same error
    assert c.params() == -2
    c.close()


def test_call_order_errors(H):
    c = FakeCtx(H)
    L = H.lib()
    assert L.hlb_step(c.ctx, 1) == -5          # no fields yet
    c.close()
    c = FakeCtx(H)
    assert c.params() == 0
    assert L.hlb_step(c.ctx, -1) == -1
    c.close()
    c = FakeCtx(H)
    assert c.params() == 0
    assert L.hlb_get_totals(c.ctx, None, None, None) == -5
    assert L.hlb_state_bytes(c.ctx) == 24 * 8 ** 3 * 8
    c.close()
