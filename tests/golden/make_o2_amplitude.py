"""Write tests/golden/o2_amplitude.json: the amplitude A of the double-twist
(O2) seed that minimises the oracle's total free energy on one 32^3 unit cell
at kappa = 0.7, tau = -0.5 (q0 = pi/32), by a coarse scan of A in [-0.5, 0.5]
followed by golden-section refinement.  Calls only the oracle."""
import json
import math
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_0901_3293_amd import inputs as I  # noqa: E402


def total_free_energy(p, A, cell=32):
    Q5 = I.o2_q5((cell,) * 3, p.q0, A)
    _, f, _ = oracle.chem(p, oracle.q5_to_q9(Q5))
    return oracle.psum(f)


def main():
    kappa, tau_ldg, cell = 0.7, -0.5, 32
    q = I.reduced(kappa, tau_ldg, math.pi / cell)
    p = oracle.params(**q.as_dict())
    grid = np.linspace(-0.5, 0.5, 41)
    vals = [total_free_energy(p, a, cell) for a in grid]
    k = int(np.argmin(vals))
    lo, hi = grid[max(k - 1, 0)], grid[min(k + 1, len(grid) - 1)]
    r = (math.sqrt(5) - 1) / 2
    c, d = hi - r * (hi - lo), lo + r * (hi - lo)
    fc, fd = total_free_energy(p, c, cell), total_free_energy(p, d, cell)
    while hi - lo > 1e-10:
        if fc < fd:
            hi, d, fd = d, c, fc
            c = hi - r * (hi - lo)
            fc = total_free_energy(p, c, cell)
        else:
            lo, c, fc = c, d, fd
            d = lo + r * (hi - lo)
            fd = total_free_energy(p, d, cell)
    A = 0.5 * (lo + hi)
    out = {"A": A, "kappa": kappa, "tau": tau_ldg, "cell": cell, "q0": math.pi / cell,
           "free_energy_per_site": total_free_energy(p, A, cell) / cell ** 3,
           "source": "oracle total free energy, golden section"}
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "o2_amplitude.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print(out)


if __name__ == "__main__":
    main()
