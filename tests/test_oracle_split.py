"""Pins of the oracle's split coupling (Sec. 2.2, Eqs. (17)-(21)): the
symmetric xi-stress in the second moment of the equilibrium, the body force
b = div tau - H:grad Q.

Each checks what the paper and the mathematics fix: the continuum limit of
both split terms, the moments the equilibrium and forcing must have
(Eqs. (17)-(19)), the momentum budget of a coupled step, and the property
the split is made for: at a discrete equilibrium (H = 0) the fluid stays at
rest, while the whole-stress force drives spurious velocities."""
import numpy as np
import pytest

from paper_0901_3293_amd import inputs as I
from tests import continuum as C


def P(orc, **kw):
    base = dict(tau=2.5, rho0=1.0, A0=0.01, gamma=3.0, K=0.0, q0=0.0, Gamma=0.3, xi=0.7, flow=True,
                coupling="split")
    base.update(kw)
    return orc.params(**base)


FINE = 64


@pytest.fixture(scope="module")
def smooth():
    return I.smooth_field((FINE,) * 3, amp=0.15, seed=7, modes=3)


def test_split_terms_continuum_limit(orc, smooth):
    """sigma^xi and b converge at second order to the continuum terms of
    Eqs. (7), (8) and (21) (H by Euler-Lagrange, spectral derivatives)."""
    K, q0, xi = 0.05, 1.5, 0.7
    sigc, bc = C.split_terms(smooth, A0=0.01, gamma=3.0, K=K, q0=q0, xi=xi)
    eb, es = [], []
    for L in (16, 32, 64):
        s = FINE // L
        h = 2 * np.pi / L
        Q5 = np.ascontiguousarray(smooth[:, ::s, ::s, ::s])
        p = P(orc, K=K / h ** 2, q0=q0 * h, xi=xi)
        sig, b = orc.split(p, orc.q5_to_q9(Q5))
        rb, rs = bc[:, ::s, ::s, ::s], sigc[:, :, ::s, ::s, ::s]
        eb.append(np.abs(b / h - rb).max() / np.abs(rb).max())
        es.append(np.abs(sig.reshape(rs.shape) - rs).max() / np.abs(rs).max())
    assert eb[2] < 2e-2 and es[2] < 5e-3
    assert 3.6 < eb[0] / eb[1] < 4.3 and 3.6 < eb[1] / eb[2] < 4.3
    assert 3.8 < es[0] / es[1] < 4.2 and 3.8 < es[1] / es[2] < 4.2


def _pulled(g, e):
    """g~_i(x) = g_i(x - e_i) on the periodic lattice ([i][z][y][x])."""
    return np.stack([np.roll(g[i], shift=(e[i, 2], e[i, 1], e[i, 0]), axis=(0, 1, 2)) for i in range(len(e))])


def _moments(g, e):
    ef = e.astype(float)
    m0 = g.sum(0)
    m1 = np.einsum("izyx,ia->azyx", g, ef)
    m2 = np.einsum("izyx,ia,ib->abzyx", g, ef, ef)
    return m0, m1, m2


def test_equilibrium_carries_the_stress(orc):
    """tau = 1, no force: the post-collision populations are the equilibrium
    of the pulled moments, whose second moment is rho/3 I + rho u u - sigma
    (Eq. (17)) for any symmetric sigma, including its trace; mass and
    momentum are those pulled in."""
    rng = np.random.default_rng(31)
    shape = (6, 5, 4)
    nx, ny, nz = shape
    p = P(orc, tau=1.0)
    e, w = orc.lattice()
    g = 1e-2 * rng.standard_normal((19, nz, ny, nx))
    S = rng.standard_normal((3, 3, nz, ny, nx)) * 1e-3
    sig = S + np.swapaxes(S, 0, 1)
    b = np.zeros((3, nz, ny, nx))
    gn, rho, u = orc.lb_split(p, g, b, sig.reshape(9, nz, ny, nx))
    m0, m1, m2 = _moments(_pulled(g, e), e)
    rho_ref = p.rho0 + m0
    u_ref = m1 / rho_ref
    n0, n1, n2 = _moments(gn, e)
    d = np.eye(3)[:, :, None, None, None]
    expect2 = (rho_ref - p.rho0) / 3 * d + rho_ref * u_ref[:, None] * u_ref[None, :] - sig
    assert np.abs(rho - rho_ref).max() < 1e-15 and np.abs(u - u_ref).max() < 1e-15
    assert np.abs(n0 - m0).max() < 1e-15
    assert np.abs(n1 - m1).max() < 1e-15
    assert np.abs(n2 - expect2).max() < 1e-15


def test_coupled_split_step_moments(orc):
    """One coupled step with tau = 1 (Eqs. (17)-(19)): the stored post-collision
    populations have zeroth moment rho - rho0, first moment rho u + b/2 and
    second moment rho/3 I + rho u u - sigma^xi + (u b + b u)/2 with
    u = (j + b/2)/rho of the pulled populations, sigma^xi and b from Q^n."""
    rng = np.random.default_rng(32)
    shape = (8, 7, 6)
    nx, ny, nz = shape
    p = P(orc, tau=1.0, K=0.02, q0=0.3)
    e, _ = orc.lattice()
    Q5 = I.helix_q5(shape, 0.3, 0.4, "y") + rng.uniform(-0.02, 0.02, size=(5, nz, ny, nx))
    u0 = rng.uniform(-1e-3, 1e-3, size=(3, nz, ny, nx))
    rho0 = 1 + rng.uniform(-1e-3, 1e-3, size=(nz, ny, nx))
    st = orc.State(p, Q5, u0, rho0)
    g_before = st.g.copy()
    sig, b = orc.split(p, st.Q9)
    st.step(1)
    m0, m1, _ = _moments(_pulled(g_before, e), e)
    rho = p.rho0 + m0
    u = (m1 + 0.5 * b) / rho
    n0, n1, n2 = _moments(st.g, e)
    d = np.eye(3)[:, :, None, None, None]
    sig = sig.reshape(3, 3, nz, ny, nx)
    expect2 = ((rho - p.rho0) / 3 * d + rho * u[:, None] * u[None, :] - sig
               + 0.5 * (u[:, None] * b[None, :] + b[:, None] * u[None, :]))
    assert np.abs(sig).max() > 1e-5 and np.abs(b).max() > 1e-6
    assert np.abs(n0 - m0).max() < 1e-15
    assert np.abs(n1 - (rho * u + 0.5 * b)).max() < 1e-15
    assert np.abs(n2 - expect2).max() < 1e-14


def test_split_momentum_budget(orc):
    """The stress term of the equilibrium carries no mass or momentum: over
    LB steps with fixed non-uniform b and sigma, total mass is constant and
    the total bare momentum grows by exactly sum_x b per step."""
    rng = np.random.default_rng(33)
    shape = (6, 6, 5)
    nx, ny, nz = shape
    p = P(orc)
    e, _ = orc.lattice()
    g = orc.init_g(p, np.full((nz, ny, nx), 1.0), np.zeros((3, nz, ny, nx)))
    S = rng.standard_normal((3, 3, nz, ny, nx)) * 1e-3
    sig = (S + np.swapaxes(S, 0, 1)).reshape(9, nz, ny, nx)
    b = rng.standard_normal((3, nz, ny, nx)) * 1e-5
    B = b.sum((1, 2, 3))
    for n in range(1, 6):
        g, _, _ = orc.lb_split(p, g, b, sig)
        m0, m1, _ = _moments(g, e)
        assert abs(m0.sum()) < 1e-15
        assert np.abs(m1.sum((1, 2, 3)) - n * B).max() < 1e-15


def test_split_coupling_has_no_spurious_velocity(orc):
    """The point of the split (Sec. 2.2): relax a double-twist (O2) lattice of
    one 16^3 unit cell with the flow off until H vanishes to rounding, then
    couple the fluid.  The split force and stress are proportional to H, so
    the fluid stays at rest to rounding; the whole-stress force, whose
    discrete divergence matches -H:grad Q only to second order, drives a
    spurious flow."""
    p0, Q, _, _ = I.bpii_case(n=16, cell=16, kappa=0.7, tau_ldg=-0.5)
    kw = dict(tau=p0.tau, rho0=p0.rho0, A0=p0.A0, gamma=p0.gamma, K=p0.K, q0=p0.q0, xi=p0.xi)
    # relaxation only: a larger Gamma reaches the same fixed point sooner (12 Gamma K = 0.22)
    st = orc.State(P(orc, Gamma=5.0, flow=False, **kw), Q)
    st.step(3000)
    Qr, _, _ = st.fields()
    H9, _, _ = orc.chem(P(orc, **kw), orc.q5_to_q9(Qr))
    assert np.abs(H9).max() < 1e-12
    umax = {}
    for c in ("force", "split"):
        s2 = orc.State(P(orc, coupling=c, **kw), Qr)
        s2.step(50)
        _, u, _ = s2.fields()
        umax[c] = np.abs(u).max()
    assert umax["force"] > 1e-7
    assert umax["split"] < 1e-12
