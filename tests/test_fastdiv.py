"""The site-index division of the kernels: floor(n / d) as a multiply-high,
an addition and a shift with m = floor(2^32 (2^l - d) / d) + 1 and
l = ceil(log2 d) (Granlund and Montgomery, 1994), computed in 32-bit unsigned
arithmetic as on the device.  Checked against integer division for every
divisor up to 4096 (and lattice-sized ones beyond) over dividends that cover
small values, every multiple boundary near the top of the range, and the
largest site index a lattice may have (n < 2^31)."""
import numpy as np

MASK = (1 << 32) - 1


def magic(d):
    l = 0
    while (1 << l) < d:
        l += 1
    m = ((1 << 32) * ((1 << l) - d)) // d + 1
    assert 0 < m <= MASK
    return m, l


def fastdiv(n, m, l):
    """The device sequence: umulhi(n, m), a 32-bit add, a shift."""
    t = (n * m) >> 32
    s = t + n
    assert s <= MASK  # the 32-bit sum does not wrap for n < 2^31
    return s >> l


def dividends(d, rng):
    top = (1 << 31) - 1
    k = top // d
    ns = set(range(0, min(4 * d + 3, 1 << 14)))
    for j in (k - 2, k - 1, k):
        for e in (-1, 0, 1):
            v = j * d + e
            if 0 <= v <= top:
                ns.add(v)
    ns.update({top, top - 1, (1 << 30), (1 << 30) - 1})
    ns.update(int(x) for x in rng.integers(0, top + 1, size=256))
    return sorted(ns)


def test_fastdiv_exact_small_divisors():
    rng = np.random.default_rng(0)
    for d in range(1, 4097):
        m, l = magic(d)
        for n in dividends(d, rng):
            assert fastdiv(n, m, l) == n // d, (n, d)


def test_fastdiv_exact_lattice_divisors():
    """Divisors that are plane sizes (nx ny) of large lattices."""
    rng = np.random.default_rng(1)
    for d in (96 * 96, 128 * 128, 257 * 255, 770 * 770, 1000 * 999, 4099 * 4093, (1 << 20) + 7, (1 << 30) - 1):
        m, l = magic(d)
        for n in dividends(d, rng):
            assert fastdiv(n, m, l) == n // d, (n, d)


def test_fastdiv_powers_of_two_are_shifts():
    for l in range(0, 31):
        m, ll = magic(1 << l)
        assert (m, ll) == (1, l)
