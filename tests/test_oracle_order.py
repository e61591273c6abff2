"""Pins of the order/disclination oracle (Sec. 2.1 local order and threshold,
Sec. 2.3 director) to closed forms: uniaxial and biaxial tensors built from
known eigen-systems, the isotropic state, and the ordering of eigenvalues."""
import numpy as np

from oracle import order as O


def _q5(Q):
    """[..., 3, 3] -> [5][...] stored components."""
    return np.stack([Q[..., 0, 0], Q[..., 0, 1], Q[..., 0, 2], Q[..., 1, 1], Q[..., 1, 2]])


def _rotations(rng, n):
    A = rng.standard_normal((n, 3, 3))
    R, _ = np.linalg.qr(A)
    return R


def test_uniaxial_closed_form():
    """Q = S (n n - I/3): q = 2S/3, director +-n, two-fold lower eigenvalue -S/3."""
    rng = np.random.default_rng(41)
    n = rng.standard_normal((64, 3))
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    S = rng.uniform(0.05, 0.7, size=64)
    Q = S[:, None, None] * (n[:, :, None] * n[:, None, :] - np.eye(3) / 3)
    q, d, defect, gap = O.order(_q5(Q)[:, :, None, None])
    q, d, defect, gap = q[:, 0, 0], d[:, :, 0, 0], defect[:, 0, 0], gap[:, 0, 0]
    assert np.abs(q - 2 * S / 3).max() < 1e-15
    assert np.abs(np.abs(np.einsum("ai,ia->i", d, n)) - 1).max() < 1e-14
    assert np.abs(gap - S).max() < 1e-15
    assert np.array_equal(defect, 2 * S / 3 < 0.19)


def test_biaxial_closed_form():
    """Q = R diag(l) R^T with l traceless: q = max l, director = the matching
    column of R; the largest, not the smallest or middle eigenvalue."""
    rng = np.random.default_rng(42)
    m = 200
    R = _rotations(rng, m)
    a, b = rng.uniform(-0.4, 0.4, size=(2, m))
    lam = np.stack([a, b, -a - b], 1)
    Q = np.einsum("nij,nj,nkj->nik", R, lam, R)
    q, d, _, gap = O.order(_q5(Q)[:, :, None, None])
    q, d, gap = q[:, 0, 0], d[:, :, 0, 0], gap[:, 0, 0]
    k = lam.argmax(1)
    top = np.sort(lam, 1)
    assert np.abs(q - top[:, 2]).max() < 1e-15
    assert np.abs(gap - (top[:, 2] - top[:, 1])).max() < 1e-14
    ok = gap > 1e-6
    dots = np.abs(np.einsum("ni,ni->n", d.T, R[np.arange(m), :, k]))
    assert np.abs(dots[ok] - 1).max() < 1e-9


def test_isotropic_and_threshold():
    """Q = 0: q = 0, a disclination site at any positive threshold; the
    threshold is strict (q == threshold is not a defect)."""
    Q5 = np.zeros((5, 2, 2, 2))
    q, _, defect, _ = O.order(Q5)
    assert np.all(q == 0) and np.all(defect)
    S = 0.285  # 2S/3 = 0.19
    Q5 = _q5((S * (np.diag([1.0, 0, 0]) - np.eye(3) / 3))[None])[:, :, None, None]
    q1 = float(O.order(Q5)[0].ravel()[0])
    assert abs(q1 - 0.19) < 1e-15
    assert not O.order(Q5, threshold=q1)[2].any()
    assert O.order(Q5, threshold=float(np.nextafter(q1, 1.0)))[2].all()


def test_defects_per_plane_counts():
    defect = np.zeros((4, 3, 5), dtype=bool)
    defect[1, 0, :2] = True
    defect[3] = True
    assert list(O.defects_per_plane(defect)) == [0, 2, 0, 15]
