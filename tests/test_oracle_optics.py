"""Pins of the polarised-light oracle (Sec. 2.3): closed forms of a uniform
retarder between crossed and parallel polarisers, the dark state of a
director along the beam, and an independent Jones-calculus evaluation of
random multi-layer stacks (which fixes the layer order and the matrix
entries)."""
import numpy as np

from oracle import optics as OP


def _column(d_list, q_list):
    """A 1x1 column of layers with given directors and orders."""
    d = np.array(d_list, dtype=np.float64).T[:, :, None, None]
    q = np.array(q_list, dtype=np.float64)[:, None, None]
    return q, d


def _delta(q, dz, lam, n_o=OP.N_O, n_e=OP.N_E):
    s2 = 1 - dz * dz
    return 2 * np.pi * q / lam * (n_o * n_e / np.sqrt(n_o ** 2 * s2 + n_e ** 2 * dz ** 2) - n_o)


def test_uniform_stack_closed_form():
    """N equal layers, in-plane director at angle t, crossed polarisers:
    S0 = 1/2 sin^2(2t) sin^2(N delta / 2); parallel: 1/2 - that."""
    rng = np.random.default_rng(51)
    for _ in range(20):
        t = rng.uniform(0, np.pi)
        q = rng.uniform(0.1, 0.5)
        N = int(rng.integers(1, 12))
        lam = rng.uniform(10, 30)
        qq, d = _column([(np.cos(t), np.sin(t), 0.0)] * N, [q] * N)
        D = N * _delta(q, 0.0, lam)
        S = OP.stokes_out(qq, d, lam)
        assert abs(S[0, 0, 0] - 0.5 * np.sin(2 * t) ** 2 * np.sin(D / 2) ** 2) < 1e-14
        S = OP.stokes_out(qq, d, lam, phi_out=0.0)
        assert abs(S[0, 0, 0] - (0.5 - 0.5 * np.sin(2 * t) ** 2 * np.sin(D / 2) ** 2)) < 1e-14


def test_director_along_beam_is_dark():
    """d = z: no retardance; crossed polarisers extinguish, and the tilt of the
    formula's delta vanishes exactly."""
    qq, d = _column([(0.0, 0.0, 1.0)] * 5, [0.4] * 5)
    assert abs(OP.stokes_out(qq, d, 16.0)[0, 0, 0]) < 1e-17
    assert abs(OP.stokes_out(qq, d, 16.0, phi_out=0.0)[0, 0, 0] - 0.5) < 1e-16


def _jones_intensity(q, d, lam, phi_in, phi_out):
    """Intensity through polariser, retarders (layer 0 first) and analyser by
    Jones calculus, averaged over the two orthogonal polarisations of
    unpolarised light."""
    total = 0.0
    for E0 in (np.array([1.0, 0.0], complex), np.array([0.0, 1.0], complex)):
        pin = np.array([np.cos(phi_in), np.sin(phi_in)])
        E = pin * (pin @ E0)
        for k in range(q.shape[0]):
            dx, dy, dz = d[:, k, 0, 0]
            b = np.arctan2(dy, dx)
            de = _delta(q[k, 0, 0], dz, lam)
            R = np.array([[np.cos(b), -np.sin(b)], [np.sin(b), np.cos(b)]])
            J = R @ np.diag([1.0, np.exp(-1j * de)]) @ R.T
            E = J @ E
        pout = np.array([np.cos(phi_out), np.sin(phi_out)])
        E = pout * (pout @ E)
        total += 0.5 * float(np.real(np.vdot(E, E)))
    return total


def test_random_stacks_match_jones_calculus():
    rng = np.random.default_rng(52)
    for _ in range(30):
        N = int(rng.integers(2, 9))
        dv = rng.standard_normal((N, 3))
        dv /= np.linalg.norm(dv, axis=1, keepdims=True)
        qv = rng.uniform(0.05, 0.5, size=N)
        qq, d = _column(list(map(tuple, dv)), list(qv))
        lam = rng.uniform(8, 24)
        pi_, po = rng.uniform(0, np.pi, size=2)
        S = OP.stokes_out(qq, d, lam, phi_in=pi_, phi_out=po)
        assert abs(S[0, 0, 0] - _jones_intensity(qq, d, lam, pi_, po)) < 1e-13


def test_image_is_weighted_over_wavelengths():
    rng = np.random.default_rng(53)
    Q5 = rng.uniform(-0.3, 0.3, size=(5, 6, 3, 4))
    img = OP.image(Q5)
    from oracle import order as O
    q, d, _, _ = O.order(Q5)
    ref = sum(w * OP.stokes_out(q, d, lam)[0] for lam, w in zip(OP.WAVELENGTHS, OP.WEIGHTS))
    assert img.shape == (3, 4) and np.abs(img - ref).max() < 1e-16
    assert np.all(img >= -1e-15) and np.all(img <= 0.5 + 1e-15)
