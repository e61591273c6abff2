"""hlb_get_totals_noalloc: the totals reduced in the library's static device
scratch, through the C-ABI, against hlb_get_totals on the same state
(bitwise: same kernels, same reduction order), on two calls in a row whose
second context is smaller, so stale partials of the first call cannot leak
into the second."""
import math

import numpy as np
import pytest

from paper_0901_3293_amd import inputs as I
from tests.hlbtest import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    import torch

    assert torch.cuda.is_available()
    from paper_0901_3293_amd import hlb

    return hlb


def solver(H, shape, prec, seed, coupling="force"):
    rng = np.random.default_rng(seed)
    nx, ny, nz = shape
    p = I.PhysParams(K=0.02, q0=0.35, gamma=3.1, coupling=coupling)
    Q = I.smooth_field(shape, amp=0.2, seed=seed) + rng.uniform(-0.02, 0.02, size=(5, nz, ny, nx))
    u = rng.uniform(-1e-3, 1e-3, size=(3, nz, ny, nx))
    rho = 1 + rng.uniform(-1e-3, 1e-3, size=(nz, ny, nx))
    s = H.Solver(shape, prec, coupling=coupling)
    s.set_params(p)
    s.set_fields(Q, u, rho)
    s.step(3)
    return s


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_totals_match_workspace_totals(H, prec):
    cases = [((96, 80, 72), "force"), ((13, 7, 9), "split")]  # the second call is smaller
    for k, (shape, coupling) in enumerate(cases):
        say("case: noalloc totals", prec, shape, coupling, "call", k + 1)
        s = solver(H, shape, prec, seed=k + 1, coupling=coupling)
        got = s.totals(noalloc=True)
        ref = s.totals()
        say("noalloc:", got, "workspace:", ref)
        assert got[0] == ref[0] and np.array_equal(got[1], ref[1]) and got[2] == ref[2]
        assert all(math.isfinite(v) for v in (got[0], got[2], *got[1]))
        s.close()


def test_noalloc_rejects_lattice_beyond_its_scratch(H):
    """A lattice above the stated maximum (26,843,136 sites) fails before any
    GPU work, with a message naming the limit; the error is sticky."""
    s = H.Solver((300, 300, 300), "fp32")
    with pytest.raises(H.HlbError) as e:
        s.totals(noalloc=True)
    say("rejected:", e.value)
    assert "26843136" in str(e.value) and e.value.code == -6
    s.close()
