"""GPU parity of the hybrid step against the FP64 oracle, through the C-ABI.

Bars: FP64 GPU vs oracle <= 1e-12 relative per field (max|d|/max|ref|) for Q,
rho and the total free energy; for u, <= 1e-12 or 8x the spread between two
valid FP64 roundings of the oracle itself, whichever is larger (the velocity is
a small difference of much larger stresses, see tests/golden/fp64_spread.json).
FP32 (deviation populations, FP32 stencils, FP64 reductions) vs the FP64
oracle: Q <= 1e-5 relative after 1000 steps.
"""
import math

import numpy as np
import pytest

from paper_0901_3293_amd import inputs as I
from tests.hlbtest import fp64_spread, oracle_params, rel, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_0901_3293_amd import hlb

    return hlb


SCHEDS = [("sites", 0), ("tiled", 8), ("mixed", 8), ("fused", 8), ("fused-tiled", 8), ("tiled", 16)]
# one schedule per kind of stress kernel: per-site, tiled, tiled and fused with the LB step
SCHEDS_CORE = [("sites", 0), ("tiled", 8), ("fused", 8)]


def make(H, p, Q, u, rho, prec="fp64", sched=("sites", 0)):
    s = H.Solver((Q.shape[3], Q.shape[2], Q.shape[1]), prec)
    s.set_params(p)
    s.set_fields(Q, u, rho)
    s.set_schedule(*sched)
    return s


@pytest.mark.parametrize("sched", SCHEDS[:5])
def test_fp64_helix_32cubed_every_step(H, orc, sched):
    """32^3 helix (q0 = 2 pi/16, kappa = 1, tau = 0, noise 1e-4, seed 1), 100
    steps: Q, u, rho and F_total at every step, every schedule."""
    say("case: fp64 helix 32^3, 100 steps", sched)
    p, Q, u, rho = I.helix_case()
    gpu = make(H, p, Q, u, rho, sched=sched)
    ref = orc.State(oracle_params(orc, p), Q, u, rho)
    spread = fp64_spread()["u"]
    worst = {"Q": 0.0, "u": 0.0, "rho": 0.0, "F": 0.0, "u/spread": 0.0}
    for n in range(100):
        gpu.step(1)
        ref.step(1)
        Qg, ug, rg = gpu.fields()
        Qr, ur, rr = ref.fields()
        mg, momg, Fg = gpu.totals()
        mr, momr, Fr = ref.totals()
        eQ, eu, er = rel(Qg, Qr), rel(ug, ur), rel(rg, rr)
        eF = abs(Fg - Fr) / abs(Fr)
        assert eQ <= 1e-12, (n, eQ)
        assert er <= 1e-12, (n, er)
        assert eF <= 1e-12, (n, eF)
        assert eu <= max(1e-12, 8 * spread[n]), (n, eu, spread[n])
        assert abs(mg - mr) / mr <= 1e-14
        worst = {"Q": max(worst["Q"], eQ), "u": max(worst["u"], eu), "rho": max(worst["rho"], er),
                 "F": max(worst["F"], eF), "u/spread": max(worst["u/spread"], eu / spread[n])}
    say("fp64 32^3 worst relative errors:", worst)


@pytest.mark.parametrize("sched", SCHEDS[:5])
def test_fp32_helix_1000_steps(H, orc, sched):
    """FP32 form vs FP64 oracle after 1000 steps: Q within 1e-5 relative."""
    say("case: fp32 helix 32^3, 1000 steps", sched)
    p, Q, u, rho = I.helix_case()
    gpu = make(H, p, Q, u, rho, "fp32", sched)
    ref = orc.State(oracle_params(orc, p), Q, u, rho)
    gpu.step(1000)
    ref.step(1000)
    Qg, ug, rg = gpu.fields()
    Qr, ur, rr = ref.fields()
    eQ, eu, er = rel(Qg, Qr), rel(ug, ur), rel(rg, rr)
    _, _, Fg = gpu.totals()
    _, _, Fr = ref.totals()
    say(f"fp32 after 1000 steps: Q {eQ:.3e}  u {eu:.3e}  rho-1 {er:.3e}  F_total {abs(Fg - Fr) / abs(Fr):.3e}")
    assert eQ <= 1e-5


@pytest.mark.parametrize("sched", SCHEDS)
@pytest.mark.parametrize("shape", [(13, 7, 9), (37, 5, 6), (4, 4, 4), (70, 3 + 2, 11)])
def test_fp64_ragged_shapes(H, orc, shape, sched):
    """Odd, non-cubic and minimum-size lattices (several blocks plus a ragged
    tail) with a strongly perturbed state, flow coupled."""
    say("case: fp64 ragged", shape, sched)
    rng = np.random.default_rng(sum(shape))
    nx, ny, nz = shape
    p = I.PhysParams(K=0.02, q0=0.35, gamma=3.1)
    Q = I.smooth_field(shape, amp=0.2, seed=5) + rng.uniform(-0.02, 0.02, size=(5, nz, ny, nx))
    u = rng.uniform(-1e-3, 1e-3, size=(3, nz, ny, nx))
    rho = 1 + rng.uniform(-1e-3, 1e-3, size=(nz, ny, nx))
    gpu = make(H, p, Q, u, rho, sched=sched)
    ref = orc.State(oracle_params(orc, p), Q, u, rho)
    for n in (1, 4, 15):
        gpu.step(n)
        ref.step(n)
        Qg, ug, rg = gpu.fields()
        Qr, ur, rr = ref.fields()
        assert rel(Qg, Qr) <= 1e-12
        assert rel(ug, ur) <= 1e-11
        assert rel(rg, rr) <= 1e-12
        assert abs(gpu.totals()[2] - ref.totals()[2]) <= 1e-12 * abs(ref.totals()[2])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_tiled_any_chunk_depth(H, orc, prec):
    """The tiled kernels march z-chunks of any depth tz (the autotuner may pick
    a depth that fills the device's block slots, e.g. 26 or 39 planes): on a
    ragged lattice (37 x 29 x 23: no side a multiple of a tile side, a prime
    depth) tz = 1, 2, 3, 5, 7 and 23 against tz = 16 in every schedule with
    tiles, and the tiled Q update on chunks of 1, 5 and 23 planes of its own
    (hlb_set_update_chunk), 6 steps.  A site's arithmetic does not depend on where the
    chunks start, so FP64 agrees bitwise (and stays within the oracle bars).
    The FP32 plane loop is unrolled by two, and the compiler fuses
    multiply-adds differently in the copies of the plane step, so a chunk
    whose planes fall differently on them rounds a few sites differently (a
    build with contraction off agrees bitwise at every depth): FP32 is held to
    1e-6 relative, about 15 units in the last place of the largest Q
    (measured at most 1.6e-7); a staging or halo mistake at a chunk edge
    would show as a difference of the order of the field's variation."""
    shape = (37, 29, 23)
    rng = np.random.default_rng(37)
    nx, ny, nz = shape
    p = I.PhysParams(K=0.02, q0=0.35, gamma=3.1)
    Q = I.smooth_field(shape, amp=0.2, seed=8) + rng.uniform(-0.02, 0.02, size=(5, nz, ny, nx))
    u = rng.uniform(-1e-3, 1e-3, size=(3, nz, ny, nx))
    rho = 1 + rng.uniform(-1e-3, 1e-3, size=(nz, ny, nx))
    steps = 6
    ref = None
    if prec == "fp64":
        o = orc.State(oracle_params(orc, p), Q, u, rho)
        o.step(steps)
        ref = o.fields()
    for name in ("tiled", "mixed", "fused", "fused-tiled"):
        base = make(H, p, Q, u, rho, prec, (name, 16))
        base.step(steps)
        Qb, ub, rb = base.fields()
        base.close()
        runs = [(tz, 0) for tz in (1, 2, 3, 5, 7, 23)]
        if name in ("tiled", "mixed", "fused-tiled"):  # the tiled Q update on a chunk of its own
            runs += [(16, tzq) for tzq in (1, 5, 23)]
        for tz, tzq in runs:
            say(f"case: {prec} {name} tz {tz} update chunk {tzq} on 37x29x23, {steps} steps")
            g = make(H, p, Q, u, rho, prec, (name, tz))
            g.set_update_chunk(tzq)
            g.step(steps)
            Qg, ug, rg = g.fields()
            g.close()
            if prec == "fp64":
                assert np.array_equal(Qg, Qb) and np.array_equal(ug, ub) and np.array_equal(rg, rb), (name, tz, tzq)
            else:
                eQ, eu, er = rel(Qg, Qb), rel(ug, ub), rel(rg, rb)
                say(f"against tz 16: Q {eQ:.2e} u {eu:.2e} rho {er:.2e}")
                assert eQ <= 1e-6 and eu <= 1e-6 and er <= 1e-6, (name, tz, tzq, eQ, eu, er)
        if ref is not None:
            Qr, ur, rr = ref
            eQ, eu, er = rel(Qb, Qr), rel(ub, ur), rel(rb, rr)
            say(f"{name} vs oracle: Q {eQ:.2e} u {eu:.2e} rho {er:.2e}")
            assert eQ <= 1e-12 and eu <= 1e-11 and er <= 1e-12


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_fused_kernel_equals_stress_and_lb_kernels(H, prec):
    """The stress evaluated inside the LB step (k_qlb) computes the force with
    the same arithmetic as the tiled stress kernel and collides with it as the
    LB kernel does, so the fused-tiled schedule reproduces the tiled one and
    the fused schedule the tiled stress followed by the per-site Q update:
    bitwise in FP64 (30 steps, ragged 37 x 29 x 23); FP32 within 1e-6 (the
    compiler may fuse the force's last multiply-add into the collision)."""
    shape = (37, 29, 23)
    rng = np.random.default_rng(41)
    nx, ny, nz = shape
    p = I.PhysParams(K=0.02, q0=0.35, gamma=3.1)
    Q = I.smooth_field(shape, amp=0.2, seed=9) + rng.uniform(-0.02, 0.02, size=(5, nz, ny, nx))
    u = rng.uniform(-1e-3, 1e-3, size=(3, nz, ny, nx))
    rho = 1 + rng.uniform(-1e-3, 1e-3, size=(nz, ny, nx))
    out = {}
    for sched in ("tiled", "fused-tiled", "fused"):
        say(f"case: {prec} {sched} tz 5 on 37x29x23, 30 steps")
        g = make(H, p, Q, u, rho, prec, (sched, 5))
        g.step(30)
        out[sched] = g.fields()
        g.close()
    a, b = out["fused-tiled"], out["tiled"]
    if prec == "fp64":
        assert all(np.array_equal(x, y) for x, y in zip(a, b))
    else:
        assert all(rel(x, y) <= 1e-6 for x, y in zip(a, b))
    # the fused schedule's Q update is the per-site one: the same step to rounding
    tol = 1e-12 if prec == "fp64" else 1e-5
    assert all(rel(x, y) <= tol for x, y in zip(out["fused"], out["tiled"]))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_large_ragged_lattice(H, orc, prec):
    """A 2.2M-site lattice with no power-of-two side (255 x 129 x 67): the
    kernels split site indices up to 2.2M by multiply-high division by 255
    and 129 and address planes by 32-bit byte offsets; every site against
    the oracle after 3 coupled steps (FP64 bar 1e-12; FP32 form within 1e-5
    on Q)."""
    shape = (255, 129, 67)
    say("case: large ragged lattice", shape, prec)
    rng = np.random.default_rng(7)
    nx, ny, nz = shape
    p = I.PhysParams(K=0.02, q0=0.35, gamma=3.1)
    Q = I.smooth_field(shape, amp=0.2, seed=6) + rng.uniform(-0.02, 0.02, size=(5, nz, ny, nx))
    u = rng.uniform(-1e-3, 1e-3, size=(3, nz, ny, nx))
    rho = 1 + rng.uniform(-1e-3, 1e-3, size=(nz, ny, nx))
    gpu = make(H, p, Q, u, rho, prec)
    say("autotuned:", gpu.autotune(3))
    ref = orc.State(oracle_params(orc, p), Q, u, rho)
    gpu.step(3)
    ref.step(3)
    Qg, ug, rg = gpu.fields()
    Qr, ur, rr = ref.fields()
    eQ, eu, er = rel(Qg, Qr), rel(ug, ur), rel(rg, rr)
    say(f"{prec} 255x129x67: Q {eQ:.2e} u {eu:.2e} rho {er:.2e}")
    if prec == "fp64":
        assert eQ <= 1e-12 and eu <= 1e-11 and er <= 1e-12
    else:
        assert eQ <= 1e-5


@pytest.mark.parametrize("sched", SCHEDS_CORE)
def test_fp64_flow_off(H, orc, sched):
    """Pure relaxation (u == 0, populations untouched)."""
    say("case: fp64 flow off 24x20x16", sched)
    p, Q, _, _ = I.helix_case(n=24, q0=2 * math.pi / 12, flow=False)
    Q = Q[:, :16, :20, :24].copy()
    gpu = make(H, p, Q, None, None, sched=sched)
    ref = orc.State(oracle_params(orc, p), Q)
    gpu.step(30)
    ref.step(30)
    Qg, ug, rg = gpu.fields()
    Qr, ur, rr = ref.fields()
    assert rel(Qg, Qr) <= 1e-12
    assert np.abs(ug).max() == 0.0
    assert np.abs(rg - 1).max() == 0.0


@pytest.mark.parametrize("sched", SCHEDS_CORE)
def test_checkpoint_restart_bitwise(H, sched):
    say("case: checkpoint 16^3", sched)
    p, Q, u, rho = I.helix_case(n=16, q0=2 * math.pi / 8)
    a = make(H, p, Q, u, rho, sched=sched)
    a.step(20)
    snap = a.get_state()
    a.step(20)
    Qa, ua, ra = a.fields()
    b = make(H, p, np.zeros_like(Q), None, None, sched=sched)
    b.set_state(snap)
    b.step(20)
    Qb, ub, rb = b.fields()
    assert np.array_equal(Qa, Qb) and np.array_equal(ua, ub) and np.array_equal(ra, rb)


@pytest.mark.parametrize("sched", SCHEDS_CORE)
def test_deterministic(H, sched):
    say("case: determinism 20^3 fp64+fp32", sched)
    p, Q, u, rho = I.helix_case(n=20, q0=2 * math.pi / 10)
    for prec in ("fp64", "fp32"):
        runs = []
        for _ in range(2):
            s = make(H, p, Q, u, rho, prec, sched)
            s.step(25)
            runs.append((s.fields(), s.totals()))
        (f1, t1), (f2, t2) = runs
        for x, y in zip(f1, f2):
            assert np.array_equal(x, y)
        assert t1[0] == t2[0] and t1[2] == t2[2] and np.array_equal(t1[1], t2[1])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("sched", SCHEDS[:5])
def test_isotropic_rest_state_is_exact_fixed_point(H, prec, sched):
    """Q = 0, u = 0, rho = rho0 (the isotropic phase at rest) is a fixed point
    of the method: H, the stress and the force vanish, and the populations
    stay at equilibrium.  It must hold exactly (bitwise zero Q and u, rho =
    rho0) on a ragged lattice in every schedule and both precisions, the
    chiral and elastic terms switched on."""
    shape = (19, 12, 10)
    nx, ny, nz = shape
    say("case: isotropic rest state", shape, prec, sched)
    p = I.PhysParams(K=0.04, q0=0.6, gamma=2.5)
    s = make(H, p, np.zeros((5, nz, ny, nx)), np.zeros((3, nz, ny, nx)), np.full((nz, ny, nx), p.rho0), prec,
             sched)
    s.step(20)
    Qg, ug, rg = s.fields()
    assert not Qg.any() and not ug.any()
    assert np.all(rg == p.rho0)


def test_nonfinite_detected(H):
    say("case: nonfinite")
    p, Q, u, rho = I.helix_case(n=8, q0=2 * math.pi / 8)
    Q = Q.copy()
    Q[0, 3, 3, 3] = np.nan
    s = make(H, p, Q, u, rho)
    with pytest.raises(H.HlbError) as e:
        s.totals()
    assert e.value.code == -4


def test_conservation_fp32_long(H):
    """FP32 form: mass (deviation sums in FP64) and momentum stay put."""
    say("case: fp32 conservation 32^3 500 steps")
    p, Q, u, rho = I.helix_case()
    s = make(H, p, Q, u, rho, "fp32")
    m0, mom0, _ = s.totals()
    s.step(500)
    m1, mom1, _ = s.totals()
    assert abs(m1 - m0) / m0 < 1e-6
    assert np.abs(mom1 - mom0).max() < 1e-6


def test_full_size_128_fp64_every_site(H, orc):
    """The 128^3 benchmark workload in the benchmark's launch configuration
    (the schedule the autotuner picks): FP64 GPU vs the oracle on every site
    after 5 steps; then the FP32 form's conservation laws over 200 steps."""
    say("case: 128^3 O2 fp64 5 steps vs oracle")
    p, Q, u, rho = I.bpii_case(n=128)
    gpu = make(H, p, Q, u, rho)
    say("autotuned:", gpu.autotune(5))
    ref = orc.State(oracle_params(orc, p), Q, u, rho)
    gpu.step(5)
    ref.step(5)
    Qg, ug, rg = gpu.fields()
    Qr, ur, rr = ref.fields()
    eQ, eu, er = rel(Qg, Qr), rel(ug, ur), rel(rg, rr)
    Fg, Fr = gpu.totals()[2], ref.totals()[2]
    say(f"128^3 fp64: Q {eQ:.2e} u {eu:.2e} rho {er:.2e} F {abs(Fg - Fr) / abs(Fr):.2e}")
    assert eQ <= 1e-12 and eu <= 1e-10 and er <= 1e-12
    assert abs(Fg - Fr) <= 1e-12 * abs(Fr)
    del gpu
    say("case: 128^3 O2 fp32 conservation")
    s = make(H, p, Q, u, rho, "fp32")
    say("autotuned:", s.autotune(5))
    m0, mom0, _ = s.totals()
    s.step(200)
    m1, mom1, _ = s.totals()
    assert abs(m1 - m0) / m0 < 1e-6
    assert np.abs(mom1 - mom0).max() < 1e-4


def test_full_size_128_fp32_vs_fp64_1000_steps(H):
    """The 128^3 benchmark workload, both forms in the benchmark's launch
    configuration (the autotuner's schedules), 1000 steps: the FP32 form
    against the FP64 GPU run (the reference at this size, itself held to the
    oracle on every site by the test above) per field -- Q within the FP32
    bar 1e-5, rho and u reported, and the free energy within 1e-5."""
    say("case: 128^3 O2 fp32 vs fp64, 1000 steps")
    p, Q, u, rho = I.bpii_case(n=128)
    a = make(H, p, Q, u, rho, "fp64")
    say("fp64 autotuned:", a.autotune(5))
    b = make(H, p, Q, u, rho, "fp32")
    say("fp32 autotuned:", b.autotune(5))
    a.step(1000)
    b.step(1000)
    Qa, ua, ra = a.fields()
    Qb, ub, rb = b.fields()
    eQ, eu, er = rel(Qb, Qa), rel(ub, ua), rel(rb - 1.0, ra - 1.0)
    Fa, Fb = a.totals()[2], b.totals()[2]
    eF = abs(Fb - Fa) / abs(Fa)
    say(f"128^3 fp32 vs fp64 after 1000 steps: Q {eQ:.2e} u {eu:.2e} rho-1 {er:.2e} F {eF:.2e}")
    assert eQ <= 1e-5
    assert eF <= 1e-5
    assert np.isfinite(ub).all() and np.isfinite(rb).all()


@pytest.mark.parametrize("kappa", [0.5, 0.8, 1.0])
def test_slab_64x64x256_full_size(H, orc, kappa):
    """The domain-growth slab at its full size (64 x 64 x 256, O2 seed for
    z < 32 inside an x-helix, tau_LdG = 0), each chirality of the sweep:
    FP64 GPU against the oracle on every site after 10 steps, and the FP32
    form's free-energy profile f(z) (the domain-wall tracker) against the
    oracle's within the FP32 bar."""
    say("case: slab 64x64x256 kappa", kappa)
    p, Q, u, rho = I.slab_case(nx=64, ny=64, nz=256, cell=32, seed_depth=32, kappa=kappa)
    ref = orc.State(oracle_params(orc, p), Q, u, rho)
    ref.step(10)
    Qr, ur, rr = ref.fields()
    _, f, _ = orc.chem(oracle_params(orc, p), ref.Q9)
    fz_ref = np.array([orc.psum(f[z]) for z in range(f.shape[0])])
    gpu = make(H, p, Q, u, rho)
    gpu.step(10)
    Qg, ug, rg = gpu.fields()
    eQ, eu, er = rel(Qg, Qr), rel(ug, ur), rel(rg, rr)
    say(f"slab fp64: Q {eQ:.2e} u {eu:.2e} rho {er:.2e} f(z) {rel(gpu.fz(), fz_ref):.2e}")
    assert eQ <= 1e-12 and eu <= 1e-10 and er <= 1e-12
    assert rel(gpu.fz(), fz_ref) <= 1e-12
    del gpu
    s32 = make(H, p, Q, u, rho, "fp32")
    s32.autotune(3)
    s32.step(10)
    e32 = rel(s32.fz(), fz_ref)
    say(f"slab fp32 f(z) {e32:.2e}")
    assert e32 <= 1e-5


def test_autotune_keeps_state(H):
    """The autotuner's trial steps leave the state untouched."""
    say("case: autotune keeps state 24^3")
    p, Q, u, rho = I.helix_case(n=24, q0=2 * math.pi / 12)
    a = make(H, p, Q, u, rho)
    a.step(3)
    before = a.fields()
    sched = a.autotune(3)
    after = a.fields()
    say("autotuned:", sched)
    for x, y in zip(before, after):
        assert np.array_equal(x, y)
    b = make(H, p, Q, u, rho, sched=sched[:2])
    b.set_update_chunk(a.update_chunk())
    b.step(3)
    a.step(4)
    b.step(4)
    for x, y in zip(a.fields(), b.fields()):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("sched", SCHEDS[1:5])
def test_schedules_agree_fp32(H, sched):
    """Every schedule gives the per-site FP32 step to rounding."""
    say("case: schedules agree fp32 40x24x20", sched)
    p, Q, u, rho = I.helix_case(n=40, q0=2 * math.pi / 10)
    Q = Q[:, :20, :24, :40].copy()
    u, rho = u[:, :20, :24, :40].copy(), rho[:20, :24, :40].copy()
    a = make(H, p, Q, u, rho, "fp32", ("sites", 0))
    b = make(H, p, Q, u, rho, "fp32", sched)
    a.step(50)
    b.step(50)
    Qa, ua, ra = a.fields()
    Qb, ub, rb = b.fields()
    assert rel(Qb, Qa) < 1e-5 and rel(rb, ra) < 1e-6


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_free_energy_profile(H, orc, prec):
    """Plane sums of f on the domain-growth slab (O2 seed in an x-helix),
    against the oracle's free-energy density summed per plane."""
    say("case: f(z) slab 32x24x40", prec)
    p, Q, u, rho = I.slab_case(nx=32, ny=24, nz=40, cell=16, seed_depth=16)
    s = make(H, p, Q, u, rho, prec)
    s.step(5)
    fz = s.fz()
    ref = orc.State(oracle_params(orc, p), Q, u, rho)
    ref.step(5)
    _, f, _ = orc.chem(oracle_params(orc, p), ref.Q9)
    fz_ref = np.array([orc.psum(f[z]) for z in range(f.shape[0])])
    tol = 1e-12 if prec == "fp64" else 1e-5
    assert rel(fz, fz_ref) <= tol
    # the seeded blue-phase slab and the helix have different plateaus
    assert abs(fz[:8].mean() - fz[-8:].mean()) > 1e-3 * np.abs(fz).max()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("sched", [("tiled", 8), ("mixed", 8), ("fused", 8), ("fused-tiled", 8), ("tiled", 16)])
@pytest.mark.parametrize("shape", [(13, 7, 9), (37, 5, 6), (64, 16, 20)])
def test_tiled_kernels_with_nan_filled_lds(H, orc, shape, sched, prec):
    """Debug mode HLB_DEBUG_NAN_LDS: every LDS plane of the tiled kernels is
    NaN before it is staged or evaluated into, so a halo point the kernels
    never write would come out as NaN.  The results stay finite and bitwise
    equal to the run without the fills, and within the bars of the oracle
    (FP64: 1e-12; FP32: Q within 1e-5), on ragged tiles and lattices narrower
    than a tile, for both tile shapes (FP32 32 x 8, FP64 16 x 12) and both
    plane structures (one barrier per plane with double-buffered LDS, and
    the FP64 Q update's two)."""
    say("case: nan-filled LDS", shape, sched, prec)
    rng = np.random.default_rng(sum(shape) + 3)
    nx, ny, nz = shape
    p = I.PhysParams(K=0.02, q0=0.35, gamma=3.1)
    Q = I.smooth_field(shape, amp=0.2, seed=8) + rng.uniform(-0.02, 0.02, size=(5, nz, ny, nx))
    u = rng.uniform(-1e-3, 1e-3, size=(3, nz, ny, nx))
    rho = 1 + rng.uniform(-1e-3, 1e-3, size=(nz, ny, nx))
    dbg = make(H, p, Q, u, rho, prec, sched)
    dbg.set_debug(nan_lds=True)
    plain = make(H, p, Q, u, rho, prec, sched)
    dbg.step(5)
    plain.step(5)
    a, b = dbg.fields(), plain.fields()
    for x, y in zip(a, b):
        assert np.isfinite(x).all() and np.array_equal(x, y)
    ref = orc.State(oracle_params(orc, p), Q, u, rho)
    ref.step(5)
    Qr, ur, rr = ref.fields()
    if prec == "fp64":
        assert rel(a[0], Qr) <= 1e-12 and rel(a[1], ur) <= 1e-11 and rel(a[2], rr) <= 1e-12
    else:
        assert rel(a[0], Qr) <= 1e-5
    assert math.isfinite(dbg.totals()[2])
