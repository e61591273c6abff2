"""Write tests/golden/fp64_spread.json: how far two valid FP64 evaluations of
the same 32^3 helix run drift apart per step when only the rounding order
differs (the oracle built as usual vs the same source built with FMA
contraction).  The velocity is a small difference of O(1e-4) stresses, so its
relative spread sits well above 1e-12; the GPU bound for u is stated relative
to this spread.  Calls only the oracle.  `--split` writes
fp64_spread_split.json for the same run with the split coupling of Sec. 2.2;
with `--d3q15` as well, fp64_spread_split_d3q15.json for the paper's D3Q15
predictor-corrector LB.  `--batch` writes fp64_spread_batch.json: the spread
of u after 13 steps on each box of inputs.batch_parity_set() (the boxes of
the batched parity test)."""
import json
import os
import subprocess
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)


def run(libpath, nsteps, coupling, lb_model="d3q19"):
    code = f"""
import os, sys, numpy as np
os.environ['HLB_ORACLE_LIB'] = {libpath!r}
sys.path.insert(0, {ROOT!r})
import oracle
from paper_0901_3293_amd import inputs as I
p, Q, u, rho = I.helix_case()
p.coupling = {coupling!r}
p.lb_model = {lb_model!r}
st = oracle.State(oracle.params(**p.as_dict()), Q, u, rho)
for n in range({nsteps}):
    st.step(1)
    q, uu, r = st.fields()
    np.save({libpath!r} + f'.{{n}}.npy', np.concatenate([q.ravel(), uu.ravel(), r.ravel()]))
"""
    subprocess.check_call([sys.executable, "-c", code])


def main(nsteps=100, coupling="force", lb_model="d3q19"):
    import oracle
    tmp = os.path.join(ROOT, "oracle", "_spread")
    os.makedirs(tmp, exist_ok=True)
    plain = os.path.join(tmp, "plain.so")
    fma = os.path.join(tmp, "fma.so")
    src = os.path.join(ROOT, "oracle", "hlb_oracle.c")
    base = [f for f in oracle.CFLAGS if f != "-ffp-contract=off"]
    subprocess.check_call(["gcc", *oracle.CFLAGS, "-o", plain, src, "-lm"])
    subprocess.check_call(["gcc", *base, "-ffp-contract=fast", "-mfma", "-o", fma, src, "-lm"])
    run(plain, nsteps, coupling, lb_model)
    run(fma, nsteps, coupling, lb_model)
    N = 32 ** 3
    spread = {"Q": [], "u": [], "rho": []}
    for n in range(nsteps):
        a = np.load(plain + f".{n}.npy")
        b = np.load(fma + f".{n}.npy")
        for k, sl in (("Q", slice(0, 5 * N)), ("u", slice(5 * N, 8 * N)), ("rho", slice(8 * N, 9 * N))):
            spread[k].append(float(np.abs(a[sl] - b[sl]).max() / np.abs(a[sl]).max()))
    for f in os.listdir(tmp):
        os.remove(os.path.join(tmp, f))
    os.rmdir(tmp)
    out = {"workload": "32^3 helix, q0 = 2 pi/16, kappa = 1, tau = 0, noise 1e-4 seed 1, FP64, "
                       f"{coupling} coupling, {lb_model} LB",
           "what": "max|a-b|/max|a| per step between the oracle built -ffp-contract=off and "
                   "built with FMA contraction",
           "spread": spread}
    name = "fp64_spread.json" if coupling == "force" else "fp64_spread_split.json"
    if lb_model == "d3q15":
        name = f"fp64_spread_{coupling}_d3q15.json"
    with open(os.path.join(HERE, name), "w") as fh:
        json.dump(out, fh)
    print({k: (v[0], v[9], v[-1]) for k, v in spread.items()})


def run_batch(libpath, nsteps):
    code = f"""
import os, sys, numpy as np
os.environ['HLB_ORACLE_LIB'] = {libpath!r}
sys.path.insert(0, {ROOT!r})
import oracle
from paper_0901_3293_amd import inputs as I
for i, r in enumerate(I.batch_parity_set()):
    st = oracle.State(oracle.params(**r['params'].as_dict()), r['Q'], r['u'], r['rho'])
    st.step({nsteps})
    q, uu, rr = st.fields()
    np.save({libpath!r} + f'.{{i}}.npy', uu.ravel())
"""
    subprocess.check_call([sys.executable, "-c", code])


def main_batch(nsteps=13):
    import oracle
    from paper_0901_3293_amd import inputs as I
    tmp = os.path.join(ROOT, "oracle", "_spread")
    os.makedirs(tmp, exist_ok=True)
    plain = os.path.join(tmp, "plain.so")
    fma = os.path.join(tmp, "fma.so")
    src = os.path.join(ROOT, "oracle", "hlb_oracle.c")
    base = [f for f in oracle.CFLAGS if f != "-ffp-contract=off"]
    subprocess.check_call(["gcc", *oracle.CFLAGS, "-o", plain, src, "-lm"])
    subprocess.check_call(["gcc", *base, "-ffp-contract=fast", "-mfma", "-o", fma, src, "-lm"])
    run_batch(plain, nsteps)
    run_batch(fma, nsteps)
    spread = []
    for i in range(len(I.batch_parity_set())):
        a = np.load(plain + f".{i}.npy")
        b = np.load(fma + f".{i}.npy")
        den = np.abs(a).max()
        spread.append(float(np.abs(a - b).max() / den) if den > 0 else 0.0)
    for f in os.listdir(tmp):
        os.remove(os.path.join(tmp, f))
    os.rmdir(tmp)
    out = {"workload": f"inputs.batch_parity_set(), FP64, whole-stress coupling, D3Q19, {nsteps} steps",
           "what": "per box: max|u_a-u_b|/max|u_a| after the steps, between the oracle built "
                   "-ffp-contract=off and built with FMA contraction",
           "spread_u": spread}
    with open(os.path.join(HERE, "fp64_spread_batch.json"), "w") as fh:
        json.dump(out, fh)
    print(spread)


if __name__ == "__main__":
    if "--batch" in sys.argv:
        main_batch()
        sys.exit(0)
    main(coupling="split" if "--split" in sys.argv else "force",
         lb_model="d3q15" if "--d3q15" in sys.argv else "d3q19")
