"""Batched form: uneven periodic boxes with their own (kappa, tau) in one
persistent launch (and its graph replay) give, box by box, exactly the result
of a single context on that box (same per-site device code), and the full
96-box replica set runs with conservation intact."""
import math

import numpy as np
import pytest

from paper_0901_3293_amd import inputs as I
from tests.hlbtest import rel, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    import torch

    assert torch.cuda.is_available()
    from paper_0901_3293_amd import hlb

    return hlb


def small_set():
    rs = I.replica_set(n_replicas=7, sizes=(8, 12, 16, 20), seed=9)
    # one box with flow switched off and one non-cubic box
    rs[2]["params"].flow = False
    Qn = I.helix_q5((10, 6, 14), 2 * math.pi / 14, 0.4, "z") + I.noise((10, 6, 14), 1e-3, 5)
    rs.append(dict(L=None, params=I.reduced(0.8, -0.2, 2 * math.pi / 14), Q=Qn, u=None, rho=None))
    return rs


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
                                              ("phases", False, 0), ("phases", False, 2000)])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batch_matches_single_boxes(H, prec, form, local, group):
    """Every launch form: the persistent kernel with boxes kept on one XCD
    (XCD-scope release) or with the fixed mapping and device-scope fences,
    and the four phase kernels per step, with all boxes in one cache group
    or in groups of at most 2000 sites (several groups, boxes larger than
    the budget alone)."""
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
