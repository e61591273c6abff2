"""Pins of the oracle's version of the paper's own LB (Sec. 2.2): D3Q15, the
printed equilibrium polynomial and coefficients, forcing P_s b.e, and the
predictor-corrector rule of Eq. (15).

The checks are the constraints the coefficients were chosen to meet
(Eqs. (17)-(20), with the third-moment reading rho/3 sym(u delta)), the
closed-form response of a uniform state to a uniform stress, exact mass and
momentum budgets, the equilibrium as a fixed point, and the scheme's stated
property: no lattice correction to the viscosity, nu -> tau T = tau/3 at
second order in k."""
import itertools

import numpy as np
import pytest

from paper_0901_3293_amd import inputs as I


def P(orc, **kw):
    base = dict(tau=2.5, rho0=1.0, A0=0.01, gamma=3.0, K=0.0, q0=0.0, Gamma=0.3, xi=0.7, flow=True,
                lb_model="d3q15")
    base.update(kw)
    return orc.params(**base)


E15 = np.array([(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
                (1, 1, 1), (-1, -1, -1), (1, 1, -1), (-1, -1, 1), (1, -1, 1), (-1, 1, -1), (-1, 1, 1),
                (1, -1, -1)], dtype=float)


def moments(g):
    m0 = g.sum(0)
    m1 = np.einsum("izyx,ia->azyx", g, E15)
    m2 = np.einsum("izyx,ia,ib->abzyx", g, E15, E15)
    m3 = np.einsum("izyx,ia,ib,ic->abczyx", g, E15, E15, E15)
    return m0, m1, m2, m3


def test_velocity_set():
    """Rest, the six faces and the eight corners of the cube, Sec. 2.2."""
    got = {tuple(int(v) for v in e) for e in E15}
    want = {(0, 0, 0)} | {tuple(v) for v in np.vstack([np.eye(3), -np.eye(3)]).astype(int)} \
        | set(itertools.product((1, -1), repeat=3))
    assert got == want and len(E15) == 15


def test_equilibrium_moments(orc):
    """Zeroth to third moments of the printed equilibrium (T = 1/3), as
    deviations from the rest state at rho0: rho - rho0, rho u,
    (rho - rho0) T I + rho u u, rho/3 sym(u delta)."""
    rng = np.random.default_rng(61)
    p = P(orc)
    shape = (3, 4, 5)
    nx, ny, nz = shape
    rho = 1 + rng.uniform(-0.05, 0.05, size=(nz, ny, nx))
    u = rng.uniform(-0.05, 0.05, size=(3, nz, ny, nx))
    g = orc.init_g(p, rho, u)
    m0, m1, m2, m3 = moments(g)
    d = np.eye(3)[:, :, None, None, None]
    assert np.abs(m0 - (rho - 1)).max() < 1e-15
    assert np.abs(m1 - rho * u).max() < 1e-16
    assert np.abs(m2 - ((rho - 1) / 3 * d + rho * u[:, None] * u[None, :])).max() < 1e-16
    sym = (np.einsum("azyx,bc->abczyx", u, np.eye(3)) + np.einsum("bzyx,ac->abczyx", u, np.eye(3))
           + np.einsum("czyx,ab->abczyx", u, np.eye(3)))
    assert np.abs(m3 - rho / 3 * sym).max() < 1e-16


@pytest.mark.parametrize("tau", [1.0, 2.5])
def test_uniform_stress_response(orc, tau):
    """A uniform state under a uniform symmetric stress sigma: the stress term
    E_s carries exactly -(sigma - tr(sigma)/3 I) in its second moment and no
    mass or momentum, so one predictor-corrector step changes the second
    moment by (sigma - tr/3 I)(1 - 2 tau)/(2 tau^2) and nothing else."""
    rng = np.random.default_rng(62)
    p = P(orc, tau=tau)
    shape = (4, 4, 4)
    rho = np.full(shape, 1.02)
    u = np.broadcast_to(np.array([0.01, -0.02, 0.015])[:, None, None, None], (3,) + shape).copy()
    g = orc.init_g(p, rho, u)
    S = rng.standard_normal((3, 3)) * 1e-3
    sig = S + S.T
    sig9 = np.broadcast_to(sig.reshape(9, 1, 1, 1), (9,) + shape).copy()
    gn, _, _ = orc.lb_pc(p, g, None, sig9)
    a0, a1, a2, _ = moments(g)
    b0, b1, b2, _ = moments(gn)
    tl = sig - np.trace(sig) / 3 * np.eye(3)
    assert np.abs(b0 - a0).max() < 1e-16 and np.abs(b1 - a1).max() < 1e-16
    expect = tl * (1 - 2 * tau) / (2 * tau ** 2)
    assert np.abs((b2 - a2) - expect[:, :, None, None, None]).max() < 1e-16


def test_mass_and_momentum_budget(orc):
    """Non-uniform b and sigma held fixed: mass is constant and the total
    momentum grows by exactly sum_x b per step (each of the two collisions
    adds b through P_s b.e, the rule averages them)."""
    rng = np.random.default_rng(63)
    p = P(orc)
    shape = (5, 6, 4)
    nx, ny, nz = shape
    rho = 1 + rng.uniform(-0.01, 0.01, size=(nz, ny, nx))
    u = rng.uniform(-0.01, 0.01, size=(3, nz, ny, nx))
    g = orc.init_g(p, rho, u)
    S = rng.standard_normal((3, 3, nz, ny, nx)) * 1e-3
    sig9 = (S + np.swapaxes(S, 0, 1)).reshape(9, nz, ny, nx)
    b = rng.standard_normal((3, nz, ny, nx)) * 1e-5
    M0 = g.sum()
    P0 = moments(g)[1].sum((1, 2, 3))
    for n in range(1, 6):
        g, _, _ = orc.lb_pc(p, g, b, sig9)
        assert abs(g.sum() - M0) < 1e-14
        assert np.abs(moments(g)[1].sum((1, 2, 3)) - P0 - n * b.sum((1, 2, 3))).max() < 1e-15


def test_equilibrium_is_a_fixed_point(orc):
    p = P(orc)
    shape = (4, 4, 4)
    u = np.broadcast_to(np.array([0.02, 0.01, -0.03])[:, None, None, None], (3,) + shape).copy()
    g = orc.init_g(p, np.full(shape, 0.98), u)
    gn, _, _ = orc.lb_pc(p, g)
    assert np.abs(gn - g).max() < 1e-17


def test_shear_viscosity_without_lattice_correction(orc):
    """A shear wave u_x = U sin(k y) decays at nu k^2 with nu -> tau T = tau/3
    (not (tau - 1/2)/3 as for plain BGK streaming), error O(k^2)."""
    tau = 1.0
    p = P(orc, tau=tau, flow=True)
    errs = []
    for L in (16, 32, 64):
        y = np.arange(L)
        k = 2 * np.pi / L
        u = np.zeros((3, 4, L, 4))
        u[0] = 1e-6 * np.sin(k * y)[None, :, None]
        g = orc.init_g(p, np.ones((4, L, 4)), u)
        amp = []
        for _ in range(400):
            g, _, uu = orc.lb_pc(p, g)
            amp.append((uu[0, 0, :, 0] * np.sin(k * y)).sum())
        nu = -np.log((amp[399] / amp[199]) ** (1 / 200)) / k ** 2
        errs.append(abs(nu - tau / 3))
    assert errs[2] < 0.01 * tau / 3
    assert 3.6 < errs[0] / errs[1] < 4.4 and 3.6 < errs[1] / errs[2] < 4.4


def test_coupled_step_is_the_scheme(orc):
    """One coupled step of the D3Q15 form with the split coupling equals
    sigma^xi and b from Q^n, one predictor-corrector LB step, and the Heun
    update of Q with the velocity of f(t) (the coupling order of Sec. 2.2)."""
    rng = np.random.default_rng(64)
    shape = (6, 5, 7)
    nx, ny, nz = shape
    p = P(orc, K=0.02, q0=0.3, coupling="split")
    Q5 = I.helix_q5(shape, 0.3, 0.4, "y") + rng.uniform(-0.02, 0.02, size=(5, nz, ny, nx))
    u0 = rng.uniform(-1e-3, 1e-3, size=(3, nz, ny, nx))
    st = orc.State(p, Q5, u0, 1 + rng.uniform(-1e-3, 1e-3, size=(nz, ny, nx)))
    g0, Q0 = st.g.copy(), st.Q9.copy()
    st.step(1)
    sig, b = orc.split(p, Q0)
    g1, _, u = orc.lb_pc(p, g0, b, sig)
    Q1 = orc.qupdate(p, Q0, u)
    assert np.array_equal(st.g, g1)
    assert np.array_equal(st.Q9, Q1)
    assert np.abs(u).max() > 1e-5
