"""Batched form: uneven periodic boxes with their own (kappa, tau) (Sec. 2.1,
the reduced chirality and temperature) in one persistent launch (and its
graph replay) match the FP64 oracle box by box, give exactly the result of a
single context on that box (same per-site device code), and the full 96-box
replica set runs with conservation intact and matches the oracle on sampled
boxes in FP32."""
import json
import math
import os

import numpy as np
import pytest

from paper_0901_3293_amd import inputs as I
from tests.hlbtest import oracle_params, rel, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    import torch

    assert torch.cuda.is_available()
    from paper_0901_3293_amd import hlb

    return hlb


def small_set():
    return I.batch_parity_set()


def single(H, prec, r, nsteps):
    Q = r["Q"]
    s = H.Solver((Q.shape[3], Q.shape[2], Q.shape[1]), prec)
    s.set_params(r["params"])
    s.set_fields(Q, r["u"], r["rho"])
    s.set_schedule("sites", 0)
    s.step(nsteps)
    return s.fields()


def make_batch(H, prec, rs):
    shapes = [(r["Q"].shape[3], r["Q"].shape[2], r["Q"].shape[1]) for r in rs]
    b = H.Batch(shapes, prec)
    for i, r in enumerate(rs):
        b.set_params(i, r["params"])
        b.set_fields(i, r["Q"], r["u"], r["rho"])
    return b


@pytest.mark.parametrize("form,local,group", [("persistent", True, 0), ("persistent", False, 0),
                                              ("persistent", True, 2000), ("persistent", False, 2000),
                                              ("phases", False, 0), ("phases", False, 2000)])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batch_matches_single_boxes(H, prec, form, local, group):
    """Every launch form: the persistent kernel with boxes kept on one XCD
    (XCD-scope release) or with the fixed mapping and device-scope fences,
    each XCD group in one cache group or in cache groups of at most
    2000 / 8 sites (every box its own); and the four phase kernels per step,
    with all boxes in one cache group or in groups of at most 2000 sites
    (several groups, boxes larger than the budget alone)."""
    say("case: batch vs single", prec, form, "xcd-local allowed", local, "group", group)
    rs = small_set()
    b = make_batch(H, prec, rs)
    b.set_chunk(8 ** 3, 256)
    b.set_launch(form, group)
    b.set_xcd_local(local)
    b.step(7)
    b.step(6)
    went_local = b.xcd_local()
    say("grid, items:", b.info(), "xcd-local barriers:", went_local)
    assert b.launch_form() == form
    if not local:
        assert not went_local
    for i, r in enumerate(rs):
        got = b.fields(i)
        ref = single(H, prec, r, 13)
        for x, y in zip(got, ref):
            assert np.array_equal(x, y), (i, rel(x, y))


@pytest.mark.parametrize("form,group", [("persistent", 0), ("phases", 3000)])
def test_batch_graph_replay(H, form, group):
    say("case: batch graph capture/replay fp32", form, group)
    rs = small_set()
    b = make_batch(H, "fp32", rs)
    b.set_launch(form, group)
    b.capture(5)
    for _ in range(3):
        b.launch()
    b.sync()
    for i, r in enumerate(rs):
        got = b.fields(i)
        ref = single(H, "fp32", r, 15)
        for x, y in zip(got, ref):
            assert np.array_equal(x, y), i


def test_batch_autotune_keeps_state(H):
    say("case: batch autotune fp32")
    rs = small_set()
    b = make_batch(H, "fp32", rs)
    b.step(2)
    before = [b.fields(i) for i in range(len(rs))]
    picks = b.autotune(2)
    say("chunks:", picks)
    assert set(picks) == {int(np.prod(r["Q"].shape[1:])) for r in rs}
    for i in range(len(rs)):
        for x, y in zip(before[i], b.fields(i)):
            assert np.array_equal(x, y)
    b.step(3)
    for i, r in enumerate(rs):
        for x, y in zip(b.fields(i), single(H, "fp32", r, 5)):
            assert np.array_equal(x, y)


def test_replica_set_96_full_size(H):
    """The 96-box scan (sizes 24/32/48/64, kappa in [0.3, 1.2], tau in [-1, 0.5]):
    50 graph-replayed FP32 steps; mass conserved per box, three boxes checked
    bitwise against single contexts."""
    say("case: 96 replicas fp32")
    rs = I.replica_set()
    b = make_batch(H, "fp32", rs)
    say("chunks:", b.autotune(2))
    m0 = [b.totals(i)[0] for i in range(len(rs))]
    b.capture(25)
    b.launch()
    b.launch()
    b.sync()
    for i in range(len(rs)):
        m1 = b.totals(i)[0]
        assert abs(m1 - m0[i]) / m0[i] < 1e-6
    for i in (0, 17, 95):
        for x, y in zip(b.fields(i), single(H, "fp32", rs[i], 50)):
            assert np.array_equal(x, y), i


@pytest.mark.parametrize("form,local,group", [("persistent", True, 0), ("persistent", True, 2000),
                                              ("phases", False, 2000)])
def test_batch_fp64_matches_oracle(H, orc, form, local, group):
    """Every box of the uneven set -- cubes of 8 to 20 with their own (kappa,
    tau), the flow-off box and the 10 x 6 x 14 box -- against the FP64 oracle
    after 13 steps (7 + 6 in two calls): Q, rho and the total free energy
    within 1e-12 relative, mass to 1e-14; u within 8 times the spread of two
    valid FP64 roundings of the oracle itself on that box after 13 steps
    (tests/golden/fp64_spread_batch.json; the velocity is a small difference
    of much larger stresses), and exactly zero with the flow off."""
    say("case: batch fp64 vs oracle", form, "xcd-local allowed", local, "group", group)
    rs = small_set()
    b = make_batch(H, "fp64", rs)
    b.set_chunk(8 ** 3, 256)
    b.set_launch(form, group)
    b.set_xcd_local(local)
    b.step(7)
    b.step(6)
    worst = {"Q": 0.0, "u": 0.0, "rho": 0.0, "F": 0.0}
    with open(os.path.join(os.path.dirname(__file__), "golden", "fp64_spread_batch.json")) as fh:
        spread_u = json.load(fh)["spread_u"]
    assert len(spread_u) == len(rs)
    for i, r in enumerate(rs):
        ref = orc.State(oracle_params(orc, r["params"]), r["Q"], r["u"], r["rho"])
        ref.step(13)
        Qg, ug, rg = b.fields(i)
        Qr, ur, rr = ref.fields()
        mg, _, Fg = b.totals(i)
        mr, _, Fr = ref.totals()
        eQ, er, eF = rel(Qg, Qr), rel(rg, rr), abs(Fg - Fr) / abs(Fr)
        eu = rel(ug, ur) if r["params"].flow else float(np.abs(ug).max())
        say(f"box {i} {Qg.shape[1:]} flow {r['params'].flow}: Q {eQ:.1e} u {eu:.1e} rho {er:.1e} F {eF:.1e}")
        assert eQ <= 1e-12 and er <= 1e-12 and eF <= 1e-12, i
        assert eu <= (max(1e-12, 8 * spread_u[i]) if r["params"].flow else 0.0), (i, eu, spread_u[i])
        assert abs(mg - mr) / mr <= 1e-14, i
        worst = {k: max(worst[k], v) for k, v in zip(worst, (eQ, eu, er, eF))}
    say("worst:", worst)


@pytest.mark.parametrize("form", ["phases", "persistent"])
def test_replica_set_96_fp32_matches_oracle(H, orc, form):
    """The full 96-box FP32 scan for 1000 steps in 20 graph replays of 50
    steps; two boxes of it (a 24^3 and a 32^3 box with their own kappa and
    tau) against the FP64 oracle: Q within 1e-5 relative, the FP32 bar of
    the single-box form."""
    say("case: 96 replicas fp32, 1000 steps vs oracle on two boxes", form)
    rs = I.replica_set()
    picks = [next(i for i, r in enumerate(rs) if r["L"] == L) for L in (24, 32)]
    b = make_batch(H, "fp32", rs)
    b.set_launch(form, 1 << 21 if form == "phases" else 0)
    b.capture(50)
    for _ in range(20):
        b.launch()
    b.sync()
    for i in picks:
        r = rs[i]
        ref = orc.State(oracle_params(orc, r["params"]), r["Q"], r["u"], r["rho"])
        ref.step(1000)
        Qg, ug, rg = b.fields(i)
        Qr, ur, rr = ref.fields()
        eQ = rel(Qg, Qr)
        say(f"box {i} L {r['L']} kappa {r['kappa']:.3f} tau {r['tau_ldg']:.3f}: Q {eQ:.2e} "
            f"u {rel(ug, ur):.2e} rho-1 {rel(rg - 1, rr - 1):.2e}")
        assert eQ <= 1e-5, i
