"""Thin ctypes binding of the C-ABI in ``include/hlb.h``.

Argument marshalling only: every step of the method runs in the HIP kernels of
``libhlb.so``.  PyTorch supplies the device workspace (a uint8 tensor kept
alive by the solver object) and the HIP stream.  The library must have been
built (``__graft_entry__.build()``); importing this module without it raises.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np
import torch  # noqa: F401  (loads the HIP runtime the library links against)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhlb.so")

HLB_FP64, HLB_FP32 = 0, 1
SCHED_SITES, SCHED_TILED, SCHED_MIXED, SCHED_FUSED, SCHED_FUSED_TILED = 0, 1, 2, 3, 4
SCHEDULES = {"sites": SCHED_SITES, "tiled": SCHED_TILED, "mixed": SCHED_MIXED, "fused": SCHED_FUSED,
             "fused-tiled": SCHED_FUSED_TILED}
STATUS = {0: "HLB_OK", -1: "HLB_ERR_ARG", -2: "HLB_ERR_PARAM", -3: "HLB_ERR_HIP",
          -4: "HLB_ERR_NONFINITE", -5: "HLB_ERR_STATE", -6: "HLB_ERR_NOMEM"}


class HlbError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class LbParams(ctypes.Structure):
    _fields_ = [("tau", ctypes.c_double), ("rho0", ctypes.c_double), ("model", ctypes.c_int)]


LB_MODELS = {"d3q19": 0, "d3q15": 1}


def lb_model_code(p):
    """model of the C-ABI from p.lb_model ("d3q19" when absent)."""
    m = getattr(p, "lb_model", "d3q19")
    if m not in LB_MODELS:
        raise ValueError(f"lb_model {m!r}: one of {sorted(LB_MODELS)}")
    return LB_MODELS[m]


class FeParams(ctypes.Structure):
    _fields_ = [("A0", ctypes.c_double), ("gamma", ctypes.c_double), ("K", ctypes.c_double),
                ("q0", ctypes.c_double)]


class OpticsParams(ctypes.Structure):
    _fields_ = [("n_o", ctypes.c_double), ("n_e", ctypes.c_double), ("h", ctypes.c_double),
                ("phi_in", ctypes.c_double), ("phi_out", ctypes.c_double), ("n_wavelengths", ctypes.c_int),
                ("wavelength", ctypes.c_double * 8), ("weight", ctypes.c_double * 8)]


class BeParams(ctypes.Structure):
    _fields_ = [("Gamma", ctypes.c_double), ("xi", ctypes.c_double), ("flow_coupling", ctypes.c_int)]


FLOW_CODES = {"force": 1, "split": 2}
COUPLINGS = {"off": 0, **FLOW_CODES}


def flow_code(p):
    """flow_coupling of the C-ABI: 0 (flow off), 1 (whole stress as a body
    force) or 2 (split coupling), from p.flow and p.coupling ("force" when
    absent)."""
    if not p.flow:
        return 0
    c = getattr(p, "coupling", "force")
    if c not in FLOW_CODES:
        raise ValueError(f"coupling {c!r}: one of {sorted(FLOW_CODES)}")
    return FLOW_CODES[c]


_lib = None


def lib():
    """Load libhlb.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run __graft_entry__.build() first")
        L = ctypes.CDLL(LIB_PATH)
        vp, dp, I, sz = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int, ctypes.c_size_t
        L.hlb_workspace_bytes.argtypes = [I, I, I, I]
        L.hlb_workspace_bytes.restype = sz
        L.hlb_workspace_bytes_for.argtypes = [I, I, I, I, I, I]
        L.hlb_workspace_bytes_for.restype = sz
        L.hlb_create.argtypes = [I, I, I, I, vp, sz, vp, ctypes.POINTER(vp)]
        L.hlb_fe_from_reduced.argtypes = [ctypes.c_double] * 4 + [ctypes.POINTER(FeParams)]
        L.hlb_set_params.argtypes = [vp, ctypes.POINTER(LbParams), ctypes.POINTER(FeParams),
                                     ctypes.POINTER(BeParams)]
        L.hlb_set_fields.argtypes = [vp, dp, dp, dp]
        L.hlb_step.argtypes = [vp, I]
        L.hlb_get_fields.argtypes = [vp, dp, dp, dp]
        L.hlb_get_totals.argtypes = [vp, dp, dp, dp]
        L.hlb_get_totals_noalloc.argtypes = [vp, dp, dp, dp]
        L.hlb_state_bytes.argtypes = [vp]
        L.hlb_state_bytes.restype = sz
        L.hlb_get_state.argtypes = [vp, vp, sz]
        L.hlb_set_state.argtypes = [vp, vp, sz]
        L.hlb_get_fz.argtypes = [vp, dp]
        L.hlb_get_order.argtypes = [vp, ctypes.c_double, dp, dp, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L.hlb_get_optics.argtypes = [vp, ctypes.POINTER(OpticsParams), dp]
        L.hlb_set_schedule.argtypes = [vp, I, I]
        L.hlb_set_debug.argtypes = [vp, I]
        L.hlb_get_schedule.argtypes = [vp, ctypes.POINTER(I), ctypes.POINTER(I)]
        L.hlb_set_update_chunk.argtypes = [vp, I]
        L.hlb_get_update_chunk.argtypes = [vp, ctypes.POINTER(I)]
        L.hlb_autotune.argtypes = [vp, I, dp]
        L.hlb_step_timed.argtypes = [vp, I, dp, I]
        L.hlb_kernel_name.argtypes = [I]
        L.hlb_kernel_name.restype = ctypes.c_char_p
        ip = ctypes.POINTER(I)
        L.hlb_batch_workspace_bytes.argtypes = [I, ip, I]
        L.hlb_batch_workspace_bytes.restype = sz
        L.hlb_batch_create.argtypes = [I, ip, I, vp, sz, vp, ctypes.POINTER(vp)]
        L.hlb_batch_set_params.argtypes = [vp, I, ctypes.POINTER(LbParams), ctypes.POINTER(FeParams),
                                           ctypes.POINTER(BeParams)]
        L.hlb_batch_set_fields.argtypes = [vp, I, dp, dp, dp]
        L.hlb_batch_set_chunk.argtypes = [vp, I, I]
        L.hlb_batch_set_xcd_local.argtypes = [vp, I]
        L.hlb_batch_set_launch.argtypes = [vp, I, ctypes.c_longlong]
        L.hlb_batch_get_launch.argtypes = [vp, ip, ctypes.POINTER(ctypes.c_longlong)]
        L.hlb_batch_autotune.argtypes = [vp, I, ip, ip, I]
        L.hlb_batch_step.argtypes = [vp, I]
        L.hlb_batch_capture.argtypes = [vp, I]
        L.hlb_batch_launch.argtypes = [vp]
        L.hlb_batch_sync.argtypes = [vp]
        L.hlb_batch_get_fields.argtypes = [vp, I, dp, dp, dp]
        L.hlb_batch_get_totals.argtypes = [vp, I, dp, dp, dp]
        L.hlb_batch_info.argtypes = [vp, ip, ip]
        L.hlb_batch_xcd_local.argtypes = [vp, ip]
        L.hlb_batch_last_error.argtypes = [vp]
        L.hlb_batch_last_error.restype = ctypes.c_char_p
        L.hlb_batch_destroy.argtypes = [vp]
        L.hlb_batch_destroy.restype = None
        L.hlb_last_error.argtypes = [vp]
        L.hlb_last_error.restype = ctypes.c_char_p
        L.hlb_destroy.argtypes = [vp]
        L.hlb_destroy.restype = None
        _lib = L
    return _lib


def _dp(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def fe_from_reduced(kappa, tau_ldg, q0, A0=0.01):
    out = FeParams()
    rc = lib().hlb_fe_from_reduced(kappa, tau_ldg, q0, A0, ctypes.byref(out))
    if rc:
        raise HlbError(rc, "hlb_fe_from_reduced")
    return out


def workspace_bytes(nx, ny, nz, precision=HLB_FP64, lb_model=None, coupling=None):
    if lb_model is None and coupling is None:
        return lib().hlb_workspace_bytes(nx, ny, nz, precision)
    return lib().hlb_workspace_bytes_for(nx, ny, nz, precision, LB_MODELS[lb_model or "d3q19"],
                                         COUPLINGS[coupling or "force"])


class Solver:
    """One hybrid-LB context on the current CUDA/HIP device.

    ``shape`` is (nx, ny, nz); host arrays are float64 ``[c][z][y][x]``.
    """

    def __init__(self, shape, precision="fp64", device="cuda", stream=None, lb_model="d3q19",
                 coupling="force"):
        """lb_model ("d3q19" or "d3q15") and coupling ("off", "force" or
        "split") size the workspace; parameters of another model or coupling
        that need more raise HLB_ERR_NOMEM in set_params."""
        self.shape = tuple(int(n) for n in shape)
        self.prec = {"fp64": HLB_FP64, "fp32": HLB_FP32}[precision]
        L = lib()
        nbytes = L.hlb_workspace_bytes_for(*self.shape, self.prec, LB_MODELS[lb_model], COUPLINGS[coupling])
        if nbytes == 0:
            raise HlbError(-1, f"invalid lattice {self.shape}")
        self.device = torch.device(device)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        ctx = ctypes.c_void_p()
        rc = L.hlb_create(*self.shape, self.prec, ctypes.c_void_p(self.ws.data_ptr()), nbytes,
                          ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(ctx))
        if rc:
            raise HlbError(rc, "hlb_create")
        self.ctx = ctx

    @property
    def N(self):
        nx, ny, nz = self.shape
        return nx * ny * nz

    def _check(self, rc):
        if rc:
            raise HlbError(rc, lib().hlb_last_error(self.ctx).decode())

    def set_params(self, p):
        """p: any object with tau, rho0, A0, gamma, K, q0, Gamma, xi, flow."""
        lb = LbParams(p.tau, p.rho0, lb_model_code(p))
        fe = FeParams(p.A0, p.gamma, p.K, p.q0)
        be = BeParams(p.Gamma, p.xi, flow_code(p))
        self._check(lib().hlb_set_params(self.ctx, ctypes.byref(lb), ctypes.byref(fe), ctypes.byref(be)))

    def set_fields(self, Q5, u3=None, rho=None):
        nx, ny, nz = self.shape
        Q5 = np.ascontiguousarray(Q5, dtype=np.float64)
        assert Q5.shape == (5, nz, ny, nx)
        if u3 is not None:
            u3 = np.ascontiguousarray(u3, dtype=np.float64)
            assert u3.shape == (3, nz, ny, nx)
        if rho is not None:
            rho = np.ascontiguousarray(rho, dtype=np.float64)
            assert rho.shape == (nz, ny, nx)
        self._check(lib().hlb_set_fields(self.ctx, _dp(Q5), _dp(u3), _dp(rho)))

    def step(self, n=1):
        self._check(lib().hlb_step(self.ctx, int(n)))

    def set_schedule(self, schedule="sites", tz=0):
        self._check(lib().hlb_set_schedule(self.ctx, SCHEDULES[schedule], int(tz)))

    def set_debug(self, nan_lds=False):
        """nan_lds: fill the tiled kernels' LDS planes with NaN before each
        plane is staged or evaluated into them (halo-coverage testing)."""
        self._check(lib().hlb_set_debug(self.ctx, 1 if nan_lds else 0))

    def schedule(self):
        sc, tz = ctypes.c_int(), ctypes.c_int()
        self._check(lib().hlb_get_schedule(self.ctx, ctypes.byref(sc), ctypes.byref(tz)))
        name = {v: k for k, v in SCHEDULES.items()}[sc.value]
        return name, tz.value

    def set_update_chunk(self, tzq=0):
        """z-chunk of the tiled Q update when it should differ from the
        schedule's (0: the same; set_schedule resets it)."""
        self._check(lib().hlb_set_update_chunk(self.ctx, int(tzq)))

    def update_chunk(self):
        v = ctypes.c_int()
        self._check(lib().hlb_get_update_chunk(self.ctx, ctypes.byref(v)))
        return v.value

    def autotune(self, trial_steps=10):
        """Pick the fastest step schedule for this lattice and precision (the
        state is left as it was); returns (schedule, tz, ms per step)."""
        ms = np.zeros(1)
        self._check(lib().hlb_autotune(self.ctx, int(trial_steps), _dp(ms)))
        return (*self.schedule(), float(ms[0]))

    def step_timed(self, n=1):
        """Advance n steps timing every kernel with HIP events on the solver's
        stream; returns {kernel name: total milliseconds}."""
        ms = np.zeros(16)
        k = lib().hlb_step_timed(self.ctx, int(n), _dp(ms), ms.size)
        if k < 0:
            self._check(k)
        return {lib().hlb_kernel_name(i).decode(): float(ms[i]) for i in range(k)}

    def fields(self):
        nx, ny, nz = self.shape
        Q5 = np.empty((5, nz, ny, nx))
        u3 = np.empty((3, nz, ny, nx))
        rho = np.empty((nz, ny, nx))
        self._check(lib().hlb_get_fields(self.ctx, _dp(Q5), _dp(u3), _dp(rho)))
        return Q5, u3, rho

    def fz(self):
        """Plane sums of the free-energy density, one per z (FP64)."""
        out = np.zeros(self.shape[2])
        self._check(lib().hlb_get_fz(self.ctx, _dp(out)))
        return out

    def order(self, threshold=0.19, fields=True):
        """Local order of the current Q: dict with q [z][y][x] (largest
        eigenvalue), dir [3][z][y][x] (director), defect [z][y][x] (uint8,
        q < threshold), per_z (disclination sites per plane) and n_defect.
        fields=False returns the counts only."""
        nx, ny, nz = self.shape
        per_z = np.zeros(nz, dtype=np.int64)
        n = ctypes.c_longlong()
        q = np.empty((nz, ny, nx)) if fields else None
        d = np.empty((3, nz, ny, nx)) if fields else None
        f = np.empty((nz, ny, nx), dtype=np.uint8) if fields else None
        self._check(lib().hlb_get_order(self.ctx, float(threshold), _dp(q), _dp(d),
                                        None if f is None else f.ctypes.data_as(ctypes.c_void_p),
                                        per_z.ctypes.data_as(ctypes.c_void_p), ctypes.byref(n)))
        return {"q": q, "dir": d, "defect": f, "per_z": per_z, "n_defect": int(n.value)}

    def optics(self, wavelengths=(16.0, 18.0, 20.0), weights=(0.2, 0.6, 0.2), phi_in=0.0,
               phi_out=math.pi / 2, n_o=1.5, n_e=2.0, h=1.0):
        """Polarised-light texture: weighted S0 behind the analyser, [y][x]."""
        if len(wavelengths) != len(weights) or not 1 <= len(wavelengths) <= 8:
            raise ValueError("1..8 wavelengths with one weight each")
        op = OpticsParams(n_o, n_e, h, phi_in, phi_out, len(wavelengths))
        for k, (lam, w) in enumerate(zip(wavelengths, weights)):
            op.wavelength[k] = lam
            op.weight[k] = w
        nx, ny, _ = self.shape
        img = np.empty((ny, nx))
        self._check(lib().hlb_get_optics(self.ctx, ctypes.byref(op), _dp(img)))
        return img

    def totals(self, noalloc=False):
        """(mass, momentum[3], total free energy) at the current level;
        noalloc=True reduces in the library's static device scratch instead
        of the workspace (hlb_get_totals_noalloc)."""
        m = np.zeros(1)
        mom = np.zeros(3)
        f = np.zeros(1)
        fn = lib().hlb_get_totals_noalloc if noalloc else lib().hlb_get_totals
        self._check(fn(self.ctx, _dp(m), _dp(mom), _dp(f)))
        return float(m[0]), mom, float(f[0])

    def get_state(self):
        n = lib().hlb_state_bytes(self.ctx)
        buf = np.empty(n, dtype=np.uint8)
        self._check(lib().hlb_get_state(self.ctx, buf.ctypes.data_as(ctypes.c_void_p), n))
        return buf

    def set_state(self, buf):
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        self._check(lib().hlb_set_state(self.ctx, buf.ctypes.data_as(ctypes.c_void_p), buf.size))

    def close(self):
        if getattr(self, "ctx", None):
            lib().hlb_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many periodic boxes of uneven size advanced together (phase kernels or
    one persistent launch per call).

    ``shapes``: list of (nx, ny, nz).  Arrays per box are float64 [c][z][y][x].
    """

    def __init__(self, shapes, precision="fp32", device="cuda", stream=None):
        self.shapes = [tuple(int(v) for v in s) for s in shapes]
        self.n = len(self.shapes)
        self.prec = {"fp64": HLB_FP64, "fp32": HLB_FP32}[precision]
        dims = (ctypes.c_int * (3 * self.n))(*[v for s in self.shapes for v in s])
        self._dims = dims
        L = lib()
        nbytes = L.hlb_batch_workspace_bytes(self.n, dims, self.prec)
        if nbytes == 0:
            raise HlbError(-1, "invalid batch shapes")
        self.device = torch.device(device)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        # graph capture needs a stream of its own (the legacy null stream cannot
        # be captured); default priority
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        b = ctypes.c_void_p()
        rc = L.hlb_batch_create(self.n, dims, self.prec, ctypes.c_void_p(self.ws.data_ptr()), nbytes,
                                ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(b))
        if rc:
            raise HlbError(rc, "hlb_batch_create")
        self.b = b

    def _check(self, rc):
        if rc < 0:
            raise HlbError(rc, lib().hlb_batch_last_error(self.b).decode())
        return rc

    def set_params(self, i, p):
        lb = LbParams(p.tau, p.rho0, lb_model_code(p))
        fe = FeParams(p.A0, p.gamma, p.K, p.q0)
        be = BeParams(p.Gamma, p.xi, flow_code(p))
        self._check(lib().hlb_batch_set_params(self.b, i, ctypes.byref(lb), ctypes.byref(fe), ctypes.byref(be)))

    def set_fields(self, i, Q5, u3=None, rho=None):
        Q5 = np.ascontiguousarray(Q5, dtype=np.float64)
        u3 = None if u3 is None else np.ascontiguousarray(u3, dtype=np.float64)
        rho = None if rho is None else np.ascontiguousarray(rho, dtype=np.float64)
        nx, ny, nz = self.shapes[i]
        assert Q5.shape == (5, nz, ny, nx)
        self._check(lib().hlb_batch_set_fields(self.b, i, _dp(Q5), _dp(u3), _dp(rho)))

    def set_chunk(self, sites_of_box, chunk):
        self._check(lib().hlb_batch_set_chunk(self.b, int(sites_of_box), int(chunk)))

    LAUNCH_FORMS = {"persistent": 0, "phases": 1}

    def set_launch(self, form, group_sites=0):
        """'phases' (default: four kernels per step, cache groups of at most
        group_sites sites) or 'persistent' (one kernel, barriers per XCD group,
        cache groups of group_sites / 8 sites per group); 0 keeps the budget."""
        self._check(lib().hlb_batch_set_launch(self.b, self.LAUNCH_FORMS[form], int(group_sites)))

    def launch_form(self):
        v = ctypes.c_int()
        g = ctypes.c_longlong()
        self._check(lib().hlb_batch_get_launch(self.b, ctypes.byref(v), ctypes.byref(g)))
        return {0: "persistent", 1: "phases"}[v.value]

    def group_sites(self):
        v = ctypes.c_int()
        g = ctypes.c_longlong()
        self._check(lib().hlb_batch_get_launch(self.b, ctypes.byref(v), ctypes.byref(g)))
        return int(g.value)

    def set_xcd_local(self, enable=True):
        self._check(lib().hlb_batch_set_xcd_local(self.b, int(bool(enable))))

    def autotune(self, trial_steps=3):
        """{box size in sites: chosen chunk}; the states are left as they were."""
        n = 64
        sizes = (ctypes.c_int * n)()
        chunks = (ctypes.c_int * n)()
        k = self._check(lib().hlb_batch_autotune(self.b, int(trial_steps), sizes, chunks, n))
        return {sizes[j]: chunks[j] for j in range(min(k, n))}

    def step(self, n=1):
        self._check(lib().hlb_batch_step(self.b, int(n)))

    def capture(self, n):
        self._check(lib().hlb_batch_capture(self.b, int(n)))

    def launch(self):
        self._check(lib().hlb_batch_launch(self.b))

    def sync(self):
        self._check(lib().hlb_batch_sync(self.b))

    def info(self):
        g, n = ctypes.c_int(), ctypes.c_int()
        self._check(lib().hlb_batch_info(self.b, ctypes.byref(g), ctypes.byref(n)))
        return g.value, n.value

    def xcd_local(self):
        """Whether the last launch kept its phase barriers XCD-local."""
        v = ctypes.c_int()
        self._check(lib().hlb_batch_xcd_local(self.b, ctypes.byref(v)))
        return bool(v.value)

    def fields(self, i):
        nx, ny, nz = self.shapes[i]
        Q5 = np.empty((5, nz, ny, nx))
        u3 = np.empty((3, nz, ny, nx))
        rho = np.empty((nz, ny, nx))
        self._check(lib().hlb_batch_get_fields(self.b, i, _dp(Q5), _dp(u3), _dp(rho)))
        return Q5, u3, rho

    def totals(self, i):
        m, mom, f = np.zeros(1), np.zeros(3), np.zeros(1)
        self._check(lib().hlb_batch_get_totals(self.b, i, _dp(m), _dp(mom), _dp(f)))
        return float(m[0]), mom, float(f[0])

    def close(self):
        if getattr(self, "b", None):
            lib().hlb_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _nn_lib():
    L = lib()
    if not getattr(L, "_nn_ready", False):
        vp, dp, I, sz = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int, ctypes.c_size_t
        fp = ctypes.POINTER(ctypes.c_float)
        up = ctypes.POINTER(ctypes.c_uint16)
        L.hlbnn_param_count.restype = I
        L.hlbnn_input_channels.restype = I
        L.hlbnn_norm_size.restype = I
        L.hlbnn_workspace_bytes.argtypes = [I, I, I]
        L.hlbnn_workspace_bytes.restype = sz
        L.hlbnn_create.argtypes = [I, I, I, vp, sz, vp, ctypes.POINTER(vp)]
        L.hlbnn_set_params.argtypes = [vp, fp]
        L.hlbnn_get_params.argtypes = [vp, fp]
        L.hlbnn_get_grads.argtypes = [vp, fp]
        L.hlbnn_set_norm.argtypes = [vp, fp]
        L.hlbnn_get_norm.argtypes = [vp, fp]
        L.hlbnn_channel_stats.argtypes = [vp, vp, I, I, dp, dp]
        L.hlbnn_fit_norm.argtypes = [vp, vp, vp, I, ctypes.c_float, fp]
        L.hlbnn_warmup.argtypes = [vp, vp, I]
        L.hlbnn_history.argtypes = [vp, vp, fp, fp]
        L.hlbnn_inputs.argtypes = [vp, vp, fp]
        L.hlbnn_make_pair.argtypes = [vp, vp, I, vp, vp]
        L.hlbnn_predict.argtypes = [vp, vp, vp]
        L.hlbnn_jump.argtypes = [vp, vp]
        L.hlbnn_train_step.argtypes = [vp, vp, vp, ctypes.c_float, dp]
        L.hlbnn_layer_forward.argtypes = [vp, I, up, fp]
        L.hlbnn_layer_backward.argtypes = [vp, I, up, up, fp, fp]
        L.hlbnn_grad_trace.argtypes = [vp, vp, vp, up, fp, up, fp]
        L.hlbnn_last_error.argtypes = [vp]
        L.hlbnn_last_error.restype = ctypes.c_char_p
        L.hlbnn_destroy.argtypes = [vp]
        L.hlbnn_destroy.restype = None
        L.hlb_surrogate_advance.argtypes = [vp, vp, I, I, ctypes.c_double, ctypes.POINTER(I), dp]
        L._nn_ready = True
    return L


def _fp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def _up(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint16))


class Net:
    """The convolutional surrogate on one lattice (see include/hlb.h, hlbnn_*).

    Device tensors passed in are torch float32 CUDA tensors, contiguous, laid
    out [C, nz, ny, nx] (or flat with that many elements): inputs x have 18
    channels (Q, u, d1, s2), increments dq have 5."""

    def __init__(self, shape, device="cuda", stream=None):
        L = _nn_lib()
        self.shape = tuple(int(v) for v in shape)
        nbytes = L.hlbnn_workspace_bytes(*self.shape)
        if nbytes == 0:
            raise HlbError(-1, f"invalid lattice {self.shape}")
        self.device = torch.device(device)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        rc = L.hlbnn_create(*self.shape, ctypes.c_void_p(self.ws.data_ptr()), nbytes,
                            ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if rc:
            raise HlbError(rc, "hlbnn_create")
        self.h = h
        self.n_params = L.hlbnn_param_count()
        self.n_in = L.hlbnn_input_channels()
        self.n_norm = L.hlbnn_norm_size()

    @property
    def N(self):
        nx, ny, nz = self.shape
        return nx * ny * nz

    def _check(self, rc):
        if rc < 0:
            raise HlbError(rc, _nn_lib().hlbnn_last_error(self.h).decode())
        return rc

    @staticmethod
    def _ptr(t):
        assert t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()
        return ctypes.c_void_p(t.data_ptr())

    def set_params(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        assert p.size == self.n_params
        self._check(_nn_lib().hlbnn_set_params(self.h, _fp(p)))

    def params(self):
        p = np.empty(self.n_params, dtype=np.float32)
        self._check(_nn_lib().hlbnn_get_params(self.h, _fp(p)))
        return p

    def grads(self):
        p = np.empty(self.n_params, dtype=np.float32)
        self._check(_nn_lib().hlbnn_get_grads(self.h, _fp(p)))
        return p

    def set_norm(self, norm):
        v = np.ascontiguousarray(norm, dtype=np.float32)
        assert v.size == self.n_norm
        self._check(_nn_lib().hlbnn_set_norm(self.h, _fp(v)))

    def norm(self):
        v = np.empty(self.n_norm, dtype=np.float32)
        self._check(_nn_lib().hlbnn_get_norm(self.h, _fp(v)))
        return v

    def channel_stats(self, data, nch):
        """data: CUDA float32 tensor of nsamples*nch*N values."""
        ns = data.numel() // (nch * self.N)
        mean, std = np.zeros(nch), np.zeros(nch)
        self._check(_nn_lib().hlbnn_channel_stats(self.h, self._ptr(data), nch, ns, _dp(mean), _dp(std)))
        return mean, std

    def fit_norm(self, X, Y, beta):
        """Standardisation from pairs X [P, 18, N], Y [P, 5, N] (set and returned)."""
        ns = X.numel() // (self.n_in * self.N)
        assert Y.numel() == ns * 5 * self.N
        out = np.empty(self.n_norm, dtype=np.float32)
        self._check(_nn_lib().hlbnn_fit_norm(self.h, self._ptr(X), self._ptr(Y), ns, float(beta), _fp(out)))
        return out

    def warmup(self, solver, k):
        self._check(_nn_lib().hlbnn_warmup(self.h, solver.ctx, int(k)))

    def history(self, solver):
        nx, ny, nz = self.shape
        d1 = np.empty((5, nz, ny, nx), dtype=np.float32)
        s2 = np.empty((5, nz, ny, nx), dtype=np.float32)
        self._check(_nn_lib().hlbnn_history(self.h, solver.ctx, _fp(d1), _fp(s2)))
        return d1, s2

    def inputs(self, solver):
        """The raw network inputs [18, nz, ny, nx] the next jump would read."""
        nx, ny, nz = self.shape
        x = np.empty((self.n_in, nz, ny, nx), dtype=np.float32)
        self._check(_nn_lib().hlbnn_inputs(self.h, solver.ctx, _fp(x)))
        return x

    def make_pair(self, solver, k, x_out, dq_out):
        """x_out <- inputs of the solver now; k solver steps; dq_out <- Q(t+k) - Q(t)."""
        self._check(_nn_lib().hlbnn_make_pair(self.h, solver.ctx, int(k), self._ptr(x_out), self._ptr(dq_out)))

    def predict(self, x, out=None):
        if out is None:
            out = torch.empty((5,) + self.shape[::-1], dtype=torch.float32, device=self.device)
        self._check(_nn_lib().hlbnn_predict(self.h, self._ptr(x), self._ptr(out)))
        return out

    def jump(self, solver):
        self._check(_nn_lib().hlbnn_jump(self.h, solver.ctx))

    def train_step(self, x, dq, lr, want_loss=True):
        loss = np.zeros(1)
        self._check(_nn_lib().hlbnn_train_step(self.h, self._ptr(x), self._ptr(dq), float(lr),
                                                _dp(loss) if want_loss else None))
        return float(loss[0]) if want_loss else None

    def grad_trace(self, x, dq):
        """Gradient of one training step without the update, with the layer
        inputs, the last output and each layer's output gradient: returns
        (acts [4][N][32] uint16 bf16 bits, y [N][5], dz list of [N][cout_padded]
        uint16, grad)."""
        acts = np.empty((4, self.N, 32), dtype=np.uint16)
        y = np.empty((self.N, 5), dtype=np.float32)
        dz = np.zeros((4, self.N, 32), dtype=np.uint16)
        g = np.empty(_nn_lib().hlbnn_param_count(), dtype=np.float32)
        self._check(_nn_lib().hlbnn_grad_trace(self.h, self._ptr(x), self._ptr(dq), _up(acts), _fp(y), _up(dz),
                                               _fp(g)))
        dzl = [dz[l].reshape(-1)[:self.N * (16 if l == 3 else 32)].reshape(self.N, -1) for l in range(4)]
        return acts, y, dzl, g

    def layer_forward(self, layer, x_bf16):
        co = (32, 32, 32, 5)[layer]
        x = np.ascontiguousarray(x_bf16, dtype=np.uint16)
        assert x.size == self.N * 32
        z = np.empty((self.N, co), dtype=np.float32)
        self._check(_nn_lib().hlbnn_layer_forward(self.h, layer, _up(x), _fp(z)))
        return z

    def layer_backward(self, layer, x_bf16, dz_bf16):
        ci, co = (self.n_in, 32, 32, 32)[layer], (32, 32, 32, 5)[layer]
        cop = 16 if layer == 3 else 32
        x = np.ascontiguousarray(x_bf16, dtype=np.uint16)
        dz = np.ascontiguousarray(dz_bf16, dtype=np.uint16)
        assert x.size == self.N * 32 and dz.size == self.N * cop
        dx = np.empty((self.N, 32), dtype=np.float32)
        g = np.empty(co * ci * 27 + co, dtype=np.float32)
        self._check(_nn_lib().hlbnn_layer_backward(self.h, layer, _up(x), _up(dz), _fp(dx), _fp(g)))
        return dx, g

    def close(self):
        if getattr(self, "h", None):
            _nn_lib().hlbnn_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def surrogate_advance(solver, net, k=8, M=4, threshold=1e-3):
    """One surrogate cycle (M jumps of k steps, the last one checked against k
    plain steps); the network must hold a history for this solver and k
    (Net.warmup).  Returns (fell_back, residual)."""
    fb = ctypes.c_int()
    r = np.zeros(1)
    rc = _nn_lib().hlb_surrogate_advance(solver.ctx, net.h, int(k), int(M), float(threshold), ctypes.byref(fb),
                                         _dp(r))
    net._check(rc)
    return bool(fb.value), float(r[0])
