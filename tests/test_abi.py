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
    N = 32 ** 3
    # per site: populations 19+19, Q 5+5, u 3, then the model's own planes --
    # the whole stress 9 (default, 60 values), the split terms 12 (63), and
    # for the D3Q15 scheme its 15 predicted populations (75 / 78); plus the
    # reduction partials
    for prec, e in ((H.HLB_FP64, 8), (H.HLB_FP32, 4)):
        want = {(None, None): 60, ("d3q19", "off"): 60, ("d3q19", "force"): 60, ("d3q19", "split"): 63,
                ("d3q15", "force"): 75, ("d3q15", "split"): 78}
        for (model, coupling), v in want.items():
            got = H.workspace_bytes(32, 32, 32, prec, model, coupling)
            assert v * e * N <= got < v * e * N + 2 ** 20, (model, coupling, got / (e * N))
    L = H.lib()
    assert L.hlb_workspace_bytes_for(32, 32, 32, H.HLB_FP32, 2, 1) == 0
    assert L.hlb_workspace_bytes_for(32, 32, 32, H.HLB_FP32, 0, 3) == 0


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


def test_set_params_checks_workspace_for_model(H):
    """A context sized for the default model rejects parameters of a model or
    coupling that needs more planes (HLB_ERR_NOMEM, sticky); one sized with
    hlb_workspace_bytes_for accepts them."""
    L = H.lib()
    p = I.PhysParams(K=0.01, q0=0.3)
    fe = H.FeParams(p.A0, p.gamma, p.K, p.q0)
    for model, coupling, tau in ((0, 2, 2.5), (1, 1, 5.0), (1, 2, 5.0)):
        for sized in (False, True):
            n = L.hlb_workspace_bytes_for(8, 8, 8, 0, model, coupling) if sized else L.hlb_workspace_bytes(8, 8, 8, 0)
            ctx = ctypes.c_void_p()
            assert L.hlb_create(8, 8, 8, 0, ctypes.c_void_p(1 << 40), n, None, ctypes.byref(ctx)) == 0
            lb = H.LbParams(tau, p.rho0, model)
            be = H.BeParams(p.Gamma, p.xi, coupling)
            rc = L.hlb_set_params(ctx, ctypes.byref(lb), ctypes.byref(fe), ctypes.byref(be))
            assert rc == (0 if sized else -6), (model, coupling, sized, rc)
            if not sized:
                assert "hlb_workspace_bytes_for" in L.hlb_last_error(ctx).decode()
            L.hlb_destroy(ctx)


def test_noalloc_totals_reject_large_lattice_before_gpu_work(H):
    """hlb_get_totals_noalloc refuses a lattice whose reduction partials do
    not fit its static scratch (26,843,136 sites at most) before touching
    the device; the error is sticky."""
    L = H.lib()
    c = FakeCtx(H, shape=(300, 300, 300))
    assert c.rc == 0
    m = ctypes.c_double()
    assert L.hlb_get_totals_noalloc(c.ctx, ctypes.byref(m), None, None) == -6
    assert "26843136" in L.hlb_last_error(c.ctx).decode()
    assert L.hlb_get_totals_noalloc(c.ctx, ctypes.byref(m), None, None) == -6
    c.close()


def test_header_is_plain_c(tmp_path):
    """include/hlb.h is a C header: a C99 program that takes the address of
    every declared function compiles with -pedantic -Werror, links against
    libhlb.so and, on the CPU, gets the documented workspace size and the
    reduced-unit mapping (Sec. 2.1, Eqs. (9)-(10)) through it."""
    import shutil
    import subprocess

    from paper_0901_3293_amd import hlb

    cc = shutil.which("gcc")
    if cc is None:
        pytest.skip("no C compiler")
    names = sorted(declared_functions())
    src = tmp_path / "abi.c"
    src.write_text(
        "#include <stdio.h>\n#include \"hlb.h\"\n"
        "typedef void (*fn)(void);\n"
        "static const fn all[] = {" + ", ".join(f"(fn)&{n}" for n in names) + "};\n"
        "int main(void)\n{\n"
        "    hlb_fe_params fe;\n"
        "    size_t b = hlb_workspace_bytes(128, 128, 128, HLB_FP32);\n"
        "    int rc = hlb_fe_from_reduced(1.0, 0.0, 0.39269908169872414, 0.01, &fe);\n"
        "    printf(\"%zu %d %.17g %u\\n\", b, rc, fe.gamma, (unsigned)(sizeof(all) / sizeof(all[0])));\n"
        "    return 0;\n}\n")
    exe = tmp_path / "abi"
    libdir = os.path.dirname(hlb.LIB_PATH)
    subprocess.run([cc, "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror",
                    "-I" + os.path.join(ROOT, "include"), str(src), "-L" + libdir, "-lhlb",
                    "-Wl,-rpath," + libdir, "-o", str(exe)], check=True, capture_output=True, text=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    assert int(out[0]) == hlb.lib().hlb_workspace_bytes(128, 128, 128, hlb.HLB_FP32) > 0
    assert int(out[1]) == 0 and float(out[2]) == pytest.approx(3.0, rel=1e-15)
    assert int(out[3]) == len(names)
