"""Local order, director and disclination sites (Sec. 2.1, 2.3) through the
C-ABI against the FP64 oracle (numpy eigh per site).

Bars: q within 1e-14 of the site's spectral scale max|eig| (both sides are
backward-stable FP64 eigen-solvers); the director, where the two largest
eigenvalues are separated by more than 1e-6 of that scale, parallel to the
oracle's to 1e-9 (|d . d_ref|, the sign being a convention), everywhere a
unit eigenvector (residual 1e-13) with its last non-zero component positive;
defect flags bit-exact except at sites whose q lies within 1e-12 of the
threshold (none occur in these inputs); per-plane counts exact."""
import numpy as np
import pytest

from oracle import order as O
from paper_0901_3293_amd import inputs as I
from tests.hlbtest import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_0901_3293_amd import hlb

    return hlb


def solver(H, Q, prec):
    nz, ny, nx = Q.shape[1:]
    s = H.Solver((nx, ny, nz), prec)
    s.set_params(I.PhysParams(K=0.02, q0=0.3))
    s.set_fields(Q, None, None)
    return s


def special_field(shape, seed):
    """Smooth field plus noise, with planted special sites: Q = 0, uniaxial
    prolate and oblate (two-fold largest eigenvalue), diagonal, tiny."""
    nx, ny, nz = shape
    rng = np.random.default_rng(seed)
    Q = I.smooth_field(shape, amp=0.3, seed=seed) + rng.uniform(-0.05, 0.05, size=(5, nz, ny, nx))
    flat = Q.reshape(5, -1)
    N = flat.shape[1]
    picks = rng.choice(N, size=min(N, 60), replace=False)
    for j, s in enumerate(picks):
        kind = j % 5
        if kind == 0:
            flat[:, s] = 0.0
        else:
            n = rng.standard_normal(3)
            n /= np.linalg.norm(n)
            S = {1: 0.5, 2: -0.4, 3: 0.3, 4: 1e-9}[kind]
            T = S * (np.outer(n, n) - np.eye(3) / 3) if kind != 3 else np.diag([0.2, -0.05, -0.15])
            flat[:, s] = [T[0, 0], T[0, 1], T[0, 2], T[1, 1], T[1, 2]]
    return flat.reshape(Q.shape)


def check(res, Qs, threshold):
    q_ref, d_ref, f_ref, gap = O.order(Qs, threshold)
    Qf = O.full_tensor(Qs)
    scale = np.abs(np.linalg.eigvalsh(Qf)).max(-1)
    q, d, f = res["q"], res["dir"], res["defect"]
    eq = np.abs(q - q_ref)
    assert np.all(eq <= 1e-14 * scale + 1e-300), eq.max()
    sep = gap > 1e-6 * scale
    dots = np.abs(np.einsum("azyx,azyx->zyx", d, d_ref))
    assert np.all(np.abs(dots[sep] - 1) <= 1e-9)
    assert np.abs(np.einsum("azyx,azyx->zyx", d, d) - 1).max() <= 1e-14
    resid = np.linalg.norm(np.einsum("zyxab,bzyx->azyx", Qf, d) - q * d, axis=0)
    assert np.all(resid <= 1e-13 * scale + 1e-300)
    last = np.where(d[2] != 0, d[2], np.where(d[1] != 0, d[1], d[0]))
    assert np.all(last > 0)
    tie = np.abs(q_ref - threshold) <= 1e-12
    assert np.array_equal(f[~tie].astype(bool), f_ref[~tie])
    assert not tie.any()
    per_z = O.defects_per_plane(f_ref)
    assert np.array_equal(res["per_z"], per_z)
    assert res["n_defect"] == int(per_z.sum())
    return int(per_z.sum())


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("shape", [(13, 7, 9), (4, 4, 4), (40, 33, 5)])
def test_order_matches_oracle(H, shape, prec):
    say("case: order vs oracle", shape, prec)
    Q = special_field(shape, seed=sum(shape))
    s = solver(H, Q, prec)
    Qs = s.fields()[0]  # the stored state (FP32-rounded in the FP32 form)
    for thr in (0.19, 0.05):
        n = check(s.order(thr), Qs, thr)
        say("threshold", thr, "defect sites", n)


def test_order_threshold_extremes(H):
    say("case: order threshold extremes")
    Q = special_field((9, 8, 7), seed=3)
    s = solver(H, Q, "fp64")
    assert s.order(0.0, fields=False)["n_defect"] == 0  # q >= 0 for traceless Q
    assert s.order(1e9, fields=False)["n_defect"] == 9 * 8 * 7
    with pytest.raises(H.HlbError):
        s.order(float("nan"))


def test_order_o2_lattice_full_size(H):
    """The 128^3 O2 workload in the FP32 form, relaxed with the flow off
    (Gamma = 5, 6000 steps) from the analytic seed (whose order is uniformly
    low, q ~ 0.1) to a blue-phase texture: q ~ 0.37 in the bulk and a network
    of disclination lines (q < 0.19).  Every site against the oracle."""
    say("case: order 128^3 O2 fp32, relaxed")
    p, Q, u, rho = I.bpii_case(n=128)
    s = H.Solver((128, 128, 128), "fp32")
    s.set_params(I.PhysParams(**{**p.as_dict(), "Gamma": 5.0, "flow": False}))
    s.set_fields(Q, u, rho)
    s.step(6000)
    res = s.order(0.19)
    n = check(res, s.fields()[0], 0.19)
    say("defect sites", n, "of", 128 ** 3, "median q", float(np.median(res["q"])))
    assert 0 < n < 128 ** 3 // 10
