"""The step on lattices whose component planes exceed 2 GiB, through the C-ABI.

The kernels address a plane of one component (N values) by 32-bit byte
offsets from its base, so offsets pass 2^31 once N exceeds 2^28 sites in FP64
or 2^29 in FP32 (the ceilings are 2^29 - 1 and 2^30 - 1 sites).  Such a
lattice is built by tiling a periodic 40^3 cell -- a cholesteric helix of
pitch 40 along z with seeded noise, repeated whole, so the big lattice is
periodic with the cell's period.  By translation symmetry every site of the
big lattice then equals the cell's site exactly after any number of steps:
the arithmetic at a site is the same, only the indexing (offsets, the
multiply-high split of the site index, the tile and block decomposition)
differs.  The cell itself is held to the FP64 oracle (Q and rho within 1e-12,
u within 1e-11 as in the ragged-lattice test over a few steps; the FP32 form
within 1e-5 on Q), so the big lattice inherits that parity site by site."""
import math

import numpy as np
import pytest

from paper_0901_3293_amd import inputs as I
from tests.hlbtest import oracle_params, rel, say

pytestmark = pytest.mark.gpu

CELL = 40
STEPS = 3


@pytest.fixture(scope="module")
def H():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_0901_3293_amd import hlb

    return hlb


def cell_case():
    p = I.reduced(1.0, 0.0, 2.0 * math.pi / CELL)
    shape = (CELL, CELL, CELL)
    Q = I.helix_q5(shape, p.q0, I.uniaxial_amplitude(p.gamma), "z") + I.noise(shape, 1e-3, 11)
    return p, Q


def equal_to_cell(big, small, reps):
    """Every site of `big` [c][z][y][x] equals `small` at the same position
    modulo the cell (bitwise)."""
    rx, ry, rz = reps
    ok = True
    for k in range(big.shape[0]):
        b = big[k].reshape(rz, CELL, ry, CELL, rx, CELL)
        ok &= bool(np.array_equal(b, np.broadcast_to(small[k][None, :, None, :, None, :], b.shape)))
    return ok


SCHEDS_LARGE = (("sites", 0), ("tiled", 32), ("fused-tiled", 32))


@pytest.mark.parametrize("prec,reps,scheds", [
    ("fp64", (16, 16, 17), SCHEDS_LARGE),   # 640 x 640 x 680 = 278.5M sites > 2^28
    ("fp32", (21, 20, 20), SCHEDS_LARGE),   # 840 x 800 x 800 = 537.6M sites > 2^29
])
def test_lattice_past_2gib_planes_equals_its_cell(H, orc, prec, reps, scheds):
    import torch

    shape = tuple(CELL * r for r in reps)
    N = shape[0] * shape[1] * shape[2]
    esz = 8 if prec == "fp64" else 4
    assert N * esz > 2 ** 31, "the case must put plane offsets past 2^31 bytes"
    need = H.workspace_bytes(*shape, {"fp64": H.HLB_FP64, "fp32": H.HLB_FP32}[prec])
    free, _ = torch.cuda.mem_get_info()
    if need > 0.9 * free:
        pytest.skip(f"needs {need / 2**30:.0f} GiB of device memory, {free / 2**30:.0f} GiB free")
    p, Qc = cell_case()

    # the cell against the oracle
    ref = orc.State(oracle_params(orc, p), Qc, None, None)
    ref.step(STEPS)
    Qr, ur, rr = ref.fields()

    big = None
    try:
        big = H.Solver(shape, prec)
        big.set_params(p)
        for sched in scheds:
            say(f"case: {prec} {shape[0]}x{shape[1]}x{shape[2]} ({N} sites, {N * esz / 2**30:.2f} GiB per plane)",
                sched)
            small = H.Solver((CELL, CELL, CELL), prec)
            small.set_params(p)
            small.set_fields(Qc)
            small.set_schedule(*sched)
            small.step(STEPS)
            Qs, us, rs = small.fields()
            small.close()
            if prec == "fp64":
                eQ, eu, er = rel(Qs, Qr), rel(us, ur), rel(rs, rr)
                say(f"cell vs oracle: Q {eQ:.2e} u {eu:.2e} rho {er:.2e}")
                assert eQ <= 1e-12 and er <= 1e-12 and eu <= 1e-11
            else:
                eQ = rel(Qs, Qr)
                say(f"cell vs oracle (FP32 form): Q {eQ:.2e}")
                assert eQ <= 1e-5

            Qb = np.tile(Qc, (1, reps[2], reps[1], reps[0]))
            big.set_fields(Qb)
            del Qb
            big.set_schedule(*sched)
            big.step(STEPS)
            torch.cuda.synchronize()
            Qg, ug, rg = big.fields()
            okQ, oku, okr = equal_to_cell(Qg, Qs, reps), equal_to_cell(ug, us, reps), \
                equal_to_cell(rg[None], rs[None], reps)
            say(f"big lattice equals its cell bitwise: Q {okQ} u {oku} rho {okr}")
            del Qg, ug, rg
            assert okQ and oku and okr
            m, _, f = big.totals()
            assert math.isfinite(m) and math.isfinite(f)
    finally:
        if big is not None:
            big.close()
        del big
        torch.cuda.empty_cache()
