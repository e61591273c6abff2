"""Throughput of the coupled hybrid-LB step on one MI355X.

Workload: the 128^3 periodic blue-phase run -- simple-cubic double-twist
(O2) initial Q of 4x4x4 unit cells of side 32 (q0 = pi/32), kappa = 0.7,
tau = -0.5, Gamma = 0.3, xi = 0.7, LB tau = 2.5, fluid at rest.  Both forms
are timed: FP32 (deviation populations, FP32 stencils) is the headline line,
FP64 is reported beside it.

Prints ONE JSON line.  MLUPS = lattice sites x steps / seconds / 1e6.  The
step time comes from HIP events on the solver's stream around exactly
`--steps` steps (after `--warmup` untimed steps), bracketed by device
synchronisation.  The roofline object is for the kernel that takes the most
time; its duration is measured in the same process with HIP events recorded
around every launch on the solver's stream.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E

# Values moved per site per launch by each kernel as scheduled (each array
# read or written once): reads + writes.  The per-site schedule's stress sweep
# writes Pi and its LB kernel reads Pi (9) instead of F (3).
KERNEL_VALUES = {
    # per-site schedule (95 values per site per step)
    "k_stress": 5 + 9,            # Q -> Pi
    "k_lb": (19 + 9) + (19 + 3),  # g, Pi -> g', u
    "k_qpred": (5 + 3) + 5,       # Q, u -> Q*
    "k_qcorr": (5 + 5 + 3) + 5,   # Q, Q*, u -> Q
    # tiled schedule (65 values per site per step)
    "k_qforce": 5 + 3,            # Q -> F
    "k_lbf": (19 + 3) + (19 + 3),  # g, F -> g', u
    "k_qupdate": (5 + 3) + 5,     # Q, u -> Q'
    # fused schedules: the stress in LDS tiles fused with the LB step (with
    # the per-site predictor and corrector 77 values per site per step, with
    # the tiled Q update 59)
    "k_qlb": 5 + 19 + (19 + 3),   # Q, g -> g', u
}
# Algorithmic values of the step of the method each kernel carries out: the
# Q-side stencil Q -> F (5 + 3), the LB step g, F -> g', u (22 + 22), the
# predictor Q, u -> Q* (8 + 5), the corrector Q, Q*, u -> Q (13 + 5), the fused
# predictor-corrector Q, u -> Q (8 + 5), the stencil fused into the LB step
# Q, g -> g', u (5 + 19 + 22).  The stress sweep of the per-site schedule is
# half of the Q-side stencil; it is counted with its own bytes.
METHOD_VALUES = {"k_lb": 44, "k_lbf": 44, "k_qforce": 8, "k_qupdate": 13, "k_qpred": 13, "k_qcorr": 18,
                 "k_stress": 14, "k_qlb": 46}
# Values per site per step of the whole step by design: four launches
# (stencil | LB | predictor | corrector), three (fused predictor-corrector),
# two (stencil fused into the LB step), and the state itself (populations and
# Q read and written once).
STEP_DESIGNS = {"4-kernel": 83, "3-kernel": 65, "2-kernel": 59, "state-minimum": 48}
# split coupling: the stress sweep writes sigma^xi (6), tau (3) and h (3)
SPLIT_VALUES = {
    "k_stress": 5 + 12,            # Q -> sigma, tau, h
    "k_lb": (19 + 12) + (19 + 3),  # g, sigma, tau, h -> g', u
}
# the paper's D3Q15 predictor-corrector LB (split coupling): two passes
PC_VALUES = {
    "k_pc1": (15 + 12) + (15 + 3 + 3),  # f, sigma/tau/h -> f + C, u, b
    "k_pc2": (15 + 15 + 6 + 3) + 15,    # f + C and f pulled, sigma, b -> f'
}

from paper_0901_3293_amd.profsum import kernel_source_sha  # noqa: E402  (hash of the step kernels' sources)


def measured_traffic(prec, kernel):
    """HBM bytes per launch of `kernel` at 128^3 from the FETCH_SIZE and
    WRITE_SIZE counter passes recorded in profiles/ (a line
    'bench-traffic: {json}' in a profile summary), if they were taken on the
    current kernel sources; None otherwise."""
    d = os.path.join(ROOT, "profiles")
    if not os.path.isdir(d):
        return None
    sha = kernel_source_sha()
    for name in sorted(os.listdir(d)):
        if not name.endswith(".md"):
            continue
        with open(os.path.join(d, name)) as fh:
            for line in fh:
                if line.startswith("bench-traffic:"):
                    rec = json.loads(line.split(":", 1)[1])
                    if rec.get("kernel_source_sha") == sha and kernel in rec.get(prec, {}):
                        return float(rec[prec][kernel]), name
    return None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def run_form(prec, n, steps, warmup, prof_steps, schedule="auto", tz=0, coupling="force", lb_model="d3q19",
             tz_update=0):
    import torch

    from paper_0901_3293_amd import hlb
    from paper_0901_3293_amd import inputs as I

    p, Q, u, rho = I.bpii_case(n=n)
    p.coupling = coupling
    p.lb_model = lb_model
    if lb_model == "d3q15":
        p.tau = 5.0  # eta = rho tau / 3 = 5/3, the viscosity of Sec. 2.1
        if coupling != "split":
            raise ValueError("the D3Q15 leg measures the paper's scheme: split coupling")
    values = {**KERNEL_VALUES, **(SPLIT_VALUES if coupling == "split" else {}), **PC_VALUES}
    s = hlb.Solver((n, n, n), prec, lb_model=lb_model, coupling=coupling)
    s.set_params(p)
    s.set_fields(Q, u, rho)
    if schedule == "auto":
        sched, tz, _ = s.autotune(40)
    else:
        s.set_schedule(schedule, tz)
        s.set_update_chunk(tz_update)
        sched, tz = s.schedule()
    tzq = s.update_chunk()
    stream = s.stream
    s.step(warmup)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    s.step(steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    kern = s.step_timed(prof_steps)
    torch.cuda.synchronize()
    m, mom, ftot = s.totals()
    esz = 4 if prec == "fp32" else 8
    N = n ** 3
    ms_step = ms / steps
    mlups = N * steps / (ms / 1e3) / 1e6
    per_launch = {k: v / prof_steps for k, v in kern.items() if v > 0}
    dom = max(per_launch, key=per_launch.get)
    alg_values = METHOD_VALUES.get(dom, values[dom]) if coupling == "force" and lb_model == "d3q19" \
        else values[dom]
    alg_bytes = alg_values * esz * N
    achieved = alg_bytes / (per_launch[dom] / 1e3) / 1e9
    step_values = sum(values[k] for k in per_launch)
    tr = measured_traffic(prec, dom) if (n == 128 and coupling == "force" and lb_model == "d3q19") else None
    gbs_of = lambda v: mlups * 1e6 * v * esz / 1e9  # noqa: E731
    out = {
        "mlups": mlups,
        "coupling": coupling,
        "lb_model": lb_model,
        "schedule": {"name": sched, "tz": tz, "tz_update": tzq},
        "ms_per_step": ms_step,
        "kernel_ms_per_launch": per_launch,
        "dominant_kernel": dom,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": tr[0] if tr else None, "traffic_source": tr[1] if tr else None,
                     "kernel": dom, "alg_values_per_site": alg_values,
                     "alg_bytes_per_launch": alg_bytes,
                     "kernel_source_sha": kernel_source_sha()},
        "step_roofline": {
            "schedule_values_per_site": step_values,
            "frac_at_schedule_values": gbs_of(step_values) / HBM_PEAK_GBS,
            **{f"frac_at_{k}_{v}": gbs_of(v) / HBM_PEAK_GBS for k, v in STEP_DESIGNS.items()},
        },
        "checks": {"mass": m, "momentum": [float(x) for x in mom], "free_energy": ftot,
                   "finite": bool(math.isfinite(m) and math.isfinite(ftot))},
    }
    s.close()
    del s
    torch.cuda.empty_cache()
    return out


def run_batched(steps, graph_steps=50, chunk=0, xcd_local=True, form=None, group=0):
    """96 uneven periodic boxes (sizes 24/32/48/64, per-box kappa and tau),
    FP32, 50-step graph replays in the autotuned launch form (or `form` with
    cache groups of `group` sites).  Aggregate MLUPS.  With
    `chunk` > 0 the autotuner is skipped and every box size uses that chunk
    (profiling runs, where every dispatch must be `graph_steps` steps)."""
    import torch

    from paper_0901_3293_amd import hlb
    from paper_0901_3293_amd import inputs as I

    rs = I.replica_set()
    shapes = [(r["L"],) * 3 for r in rs]
    b = hlb.Batch(shapes, "fp32")
    for i, r in enumerate(rs):
        b.set_params(i, r["params"])
        b.set_fields(i, r["Q"], r["u"], r["rho"])
    b.set_xcd_local(xcd_local)
    if chunk > 0:
        for L in sorted({r["L"] for r in rs}):
            b.set_chunk(L ** 3, chunk)
        chunks = {L ** 3: chunk for L in sorted({r["L"] for r in rs})}
    else:
        chunks = b.autotune(10)
    if form:
        b.set_launch(form, group)  # after the autotuner, which also picks the form
    b.capture(graph_steps)
    b.launch()
    b.sync()
    reps = max(1, steps // graph_steps)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(b.stream)
    for _ in range(reps):
        b.launch()
    ev1.record(b.stream)
    b.sync()
    ms = ev0.elapsed_time(ev1)
    sites = sum(L ** 3 for L in (r["L"] for r in rs))
    grid, items = b.info()
    xcd_local = b.xcd_local()
    masses = [b.totals(i)[0] for i in range(len(rs))]
    out = {"mlups": sites * reps * graph_steps / (ms / 1e3) / 1e6, "boxes": len(rs), "sites": sites,
           "steps": reps * graph_steps, "ms_per_step": ms / (reps * graph_steps), "grid": grid,
           "work_items": items, "launch_form": b.launch_form(), "cache_group_sites": b.group_sites(),
           "xcd_local_barriers": xcd_local,
           "chunk_by_box_sites": chunks,
           "sizes": {str(L): sum(1 for r in rs if r["L"] == L) for L in (24, 32, 48, 64)},
           "finite": bool(all(math.isfinite(m) for m in masses))}
    b.close()
    torch.cuda.empty_cache()
    return out


def run_order(n=128, calls=20, threshold=0.19, relax=6000):
    """Local order and disclination count (largest eigenvalue of Q per site,
    FP64 Jacobi) on the n^3 O2 workload in the FP32 form, relaxed first with
    the flow off (Gamma = 5, `relax` steps) from the analytic seed to a
    blue-phase texture with disclination lines: device time of a counts-only
    call (HIP events on the context's stream) and the number of disclination
    sites."""
    import numpy as np
    import torch

    from paper_0901_3293_amd import hlb
    from paper_0901_3293_amd import inputs as I

    p, Q, u, rho = I.bpii_case(n=n)
    s = hlb.Solver((n, n, n), "fp32")
    s.set_params(I.PhysParams(**{**p.as_dict(), "Gamma": 5.0, "flow": False}))
    s.set_fields(Q, u, rho)
    s.step(relax)
    res = s.order(threshold, fields=False)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t = []
    for _ in range(calls):
        ev0.record(s.stream)
        s.order(threshold, fields=False)
        ev1.record(s.stream)
        torch.cuda.synchronize()
        t.append(ev0.elapsed_time(ev1))
    ms = float(np.median(t))
    img = s.optics()
    to = []
    for _ in range(max(3, calls // 4)):
        ev0.record(s.stream)
        s.optics()
        ev1.record(s.stream)
        torch.cuda.synchronize()
        to.append(ev0.elapsed_time(ev1))
    s.close()
    torch.cuda.empty_cache()
    N = n ** 3
    return {"sites": N, "threshold": threshold, "relax_steps": relax, "n_defect": res["n_defect"],
            "optics_ms_per_call": float(np.median(to)), "optics_mean_s0": float(img.mean()),
            "ms_per_call": ms,
            "msites_per_s": N / (ms / 1e3) / 1e6,
            "note": "counts-only call: order kernel (reads 5 FP32 values, writes 1 flag byte per site), "
                    "per-plane count kernel, one small device-to-host copy"}


def run_surrogate(n=96, steps=20000, k=32, M=4, iters=3000, train_set="mixed"):
    """The surrogate workload on a 96^3 box: training pairs ("mixed": 500
    from five O2 runs and two domain-growth runs, kappa 0.7, tau -0.5, noise
    1e-3, the last run of each kind held out; "growth": 60 from each of five
    domain-growth runs after 1000 steps, one held out, and 60 from an O2 run
    for evaluation only), training on the GPU, then 20000 steps
    of the domain-growth box (O2 slab z < 32 inside an x-helix) with the
    surrogate (one network jump for k solver steps, M jumps per checked
    cycle, threshold 1e-3) against the plain FP32 form from the same state."""
    import numpy as np
    import torch

    from paper_0901_3293_amd import hlb
    from paper_0901_3293_amd import inputs as I
    from paper_0901_3293_amd import surrogate as S

    N = n ** 3
    net = hlb.Net((n, n, n))
    if train_set == "mixed":
        o2_pairs, gr_pairs, spacing, burn = 80, 50, 240, 300
        runs = ([("o2", s, o2_pairs) for s in range(4)] + [("growth", 1, gr_pairs)] +
                [("o2", 4, o2_pairs)] + [("growth", 2, gr_pairs)])
        n_train = 4 * o2_pairs + gr_pairs
    else:  # domain-growth runs only, past the early transient
        gr_pairs, spacing, burn = 60, 240, 1000
        runs = [("growth", s, gr_pairs) for s in (1, 3, 4, 5)] + [("growth", 2, gr_pairs)] + [("o2", 4, gr_pairs)]
        n_train = 4 * gr_pairs
    total = sum(r[2] for r in runs)
    pairs = S.allocate_pairs(total, N)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    slot, spans = 0, {}
    for kind, seed, count in runs:
        case = S.o2_run(n, seed=seed) if kind == "o2" else S.growth_run(n, noise_amp=1e-3, seed=seed)
        sv = S.new_solver(case)
        S.record_pairs(net, sv, pairs, slot, count, spacing, k=k, burn_in=burn, tag=f"{kind}-{seed}")
        spans[f"{kind}-{seed}"] = list(range(slot, slot + count))
        slot += count
        del sv
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    train_idx = list(range(0, n_train))
    S.fit_norm(net, pairs, 0.0, index=train_idx)
    net.set_params(I.cnn_params(seed=0))
    lr = 5e-4 if train_set == "mixed" else 1e-3
    tl = S.train(net, pairs, iters, lr=lr, index=train_idx, log_every=max(1, iters // 5))
    evals = {}
    for tag in ("o2-4", "growth-2"):
        e = S.evaluate(net, pairs, spans[tag])
        evals[tag] = {k: float(np.median(v)) for k, v in e.items()}
    # network application time (HIP events on the network's stream)
    x = pairs.X[train_idx[-1]]
    out = torch.empty((5, N), dtype=torch.float32, device="cuda")
    for _ in range(3):
        net.predict(x, out)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(net.stream)
    for _ in range(20):
        net.predict(x, out)
    e1.record(net.stream)
    torch.cuda.synchronize()
    ms_net = e0.elapsed_time(e1) / 20
    del pairs, x
    torch.cuda.empty_cache()

    case = S.growth_run(n)
    plain = S.new_solver(case)
    t_plain = S.plain_run(plain, steps)
    fz_plain = S.domain_profile(plain)
    sur = S.new_solver(case)
    st = S.run(sur, net, steps, k=k, M=M)
    fz_sur = S.domain_profile(sur)
    sweep = {}
    for m in (2 * M, 4 * M):  # jumps per checked cycle
        sv = S.new_solver(case)
        sm = S.run(sv, net, steps, k=k, M=m)
        sweep[str(m)] = {"seconds": sm.seconds, "speedup": t_plain / sm.seconds,
                         "q_error_vs_plain": S.q_error(sv, plain), "fallbacks": sm.fallbacks, "cycles": sm.cycles}
        del sv
    sv = S.new_solver(case)
    sn = S.run(sv, net, steps, k=k, M=M, refresh=None)
    no_refresh = {"seconds": sn.seconds, "speedup": t_plain / sn.seconds, "q_error_vs_plain": S.q_error(sv, plain),
                  "fallbacks": sn.fallbacks, "cycles": sn.cycles, "plain_cycles": sn.plain_cycles}
    del sv
    ex_net = hlb.Net((n, n, n))
    S.extrapolation_only(ex_net, 0.0)
    ext = S.new_solver(case)
    sx = S.run(ext, ex_net, steps, k=k, M=M)
    qx_net = hlb.Net((n, n, n))
    S.extrapolation_only(qx_net, 1.0)
    qxt = S.new_solver(case)
    sq = S.run(qxt, qx_net, steps, k=k, M=M)
    spread = float(fz_plain.max() - fz_plain.min())
    flop = 2.0 * N * S.MACS_PER_SITE
    out = {
        "workload": f"{n}^3 domain-growth box (O2 slab z<32 in an x-helix, kappa 0.7, tau -0.5), FP32, "
                    f"{steps} steps; k = {k}, M = {M}, threshold {S.THRESHOLD:g}, refresh {S.REFRESH:g}",
        "plain_fp32_s": t_plain,
        "surrogate_s": st.seconds,
        "speedup": t_plain / st.seconds,
        "q_error_vs_plain": S.q_error(sur, plain),
        "fz_max_dev_over_spread": float(np.abs(fz_sur - fz_plain).max() / spread) if spread > 0 else None,
        "domain_planes": {"plain": S.domain_size(fz_plain), "surrogate": S.domain_size(fz_sur)},
        "blue_phase_planes": {"plain": int(S.defect_walls(plain.order(fields=False)["per_z"])[0].sum()),
                              "surrogate": int(S.defect_walls(sur.order(fields=False)["per_z"])[0].sum())},
        "cycles": st.cycles, "fallbacks": st.fallbacks, "plain_cycles": st.plain_cycles,
        "fallback_steps": st.fallback_steps,
        "residual_median": float(np.median(st.residuals)) if st.residuals else None,
        "residual_max": float(np.max(st.residuals)) if st.residuals else None,
        "m_sweep": sweep,
        "without_refresh": no_refresh,
        "extrapolation_only": {"seconds": sx.seconds, "speedup": t_plain / sx.seconds,
                               "q_error_vs_plain": S.q_error(ext, plain), "fallbacks": sx.fallbacks,
                               "cycles": sx.cycles},
        "quadratic_extrapolation_only": {"seconds": sq.seconds, "speedup": t_plain / sq.seconds,
                                         "q_error_vs_plain": S.q_error(qxt, plain), "fallbacks": sq.fallbacks,
                                         "cycles": sq.cycles},
        "increment_error_heldout": evals,
        "training": {"set": train_set, "pairs": total, "train_pairs": len(train_idx), "iters": iters, "lr": lr,
                     "seconds": tl.seconds,
                     "data_seconds": t_data, "final_loss": tl.losses[-1][1] if tl.losses else None},
        "network_ms": ms_net,
        "conv_roofline": {"bound": "mfma", "achieved": flop / (ms_net * 1e-3) / 1e12, "peak": 2500.0,
                          "unit": "TFLOP/s", "frac": flop / (ms_net * 1e-3) / 1e12 / 2500.0,
                          "flop_per_site": 2 * S.MACS_PER_SITE, "kernel": "k_conv (4 layers)"},
    }
    for o in (net, ex_net, qx_net):
        o.close()
    del plain, sur, ext, qxt
    torch.cuda.empty_cache()
    return out


def run_surrogate_growth(n=96, kappa=1.0, tau_ldg=0.0, target=44, every=128, max_steps=30720, k=32, M=4,
                         iters=3000, lr=1e-3, train_seeds=(1, 3, 4, 5), heldout_seed=2, pairs_per_run=60,
                         spacing=240, burn=1000):
    """Time to a stated domain size on a growing box: an n^3 box with a
    double-twist (O2) slab z < 32 inside a cholesteric x-helix at kappa, tau
    (FP32), whose blue-phase domain (planes carrying disclination sites)
    grows.  Training pairs come from growth runs of the same box with seeded
    noise 1e-3 on Q (`pairs_per_run` per run, one every `spacing` steps after
    `burn`), one run held out; the timed runs start from the noise-free seed.
    Each predictor -- the trained network on the linear base, linear
    extrapolation alone, quadratic extrapolation alone (the driver without a
    network) -- runs in the same checked driver (k steps per jump, M jumps
    per checked cycle) and the plain FP32 step without a driver; all are read
    every `every` steps and timed (stepping only) to the first read-out at
    `target` blue-phase planes or more.  The Q error of each predictor is
    taken against the plain run at the plain run's crossing step."""
    import numpy as np
    import torch

    from paper_0901_3293_amd import hlb
    from paper_0901_3293_amd import inputs as I
    from paper_0901_3293_amd import surrogate as S

    N = n ** 3
    grow = dict(kappa=kappa, tau_ldg=tau_ldg)
    net = hlb.Net((n, n, n))
    seeds = list(train_seeds) + [heldout_seed]
    pairs = S.allocate_pairs(len(seeds) * pairs_per_run, N)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for j, seed in enumerate(seeds):
        sv = S.new_solver(S.growth_run(n, noise_amp=1e-3, seed=seed, **grow))
        S.record_pairs(net, sv, pairs, j * pairs_per_run, pairs_per_run, spacing, k=k, burn_in=burn,
                       tag=f"growth-{seed}")
        del sv
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    n_train = len(train_seeds) * pairs_per_run
    train_idx = list(range(n_train))
    held = list(range(n_train, n_train + pairs_per_run))
    S.fit_norm(net, pairs, 0.0, index=train_idx)
    net.set_params(I.cnn_params(seed=0))
    tl = S.train(net, pairs, iters, lr=lr, index=train_idx, log_every=max(1, iters // 5))
    ev = S.evaluate(net, pairs, held)
    heldout = {key: float(np.median(v)) for key, v in ev.items()}
    del pairs
    torch.cuda.empty_cache()

    case = S.growth_run(n, **grow)
    plain = S.new_solver(case)
    # the plain FP32 step at its fastest schedule; every predictor's run uses the same
    sched, tz, _ = plain.autotune(20)
    tzq = plain.update_chunk()
    T, t_plain, track_plain, _ = S.time_to_domain(plain, plain.step, target, every, max_steps)
    q_plain = plain.fields()[0] if T is not None else None
    start = track_plain[0][1] if track_plain else None
    res = {"plain": {"steps_to_target": T, "seconds": t_plain, "planes_every_read": [b for _, b in track_plain],
                     "schedule": {"name": sched, "tz": tz, "tz_update": tzq}}}
    preds = {"network": net}
    for name, beta in (("linear_extrapolation", 0.0), ("quadratic_extrapolation", 1.0)):
        e = hlb.Net((n, n, n))
        S.extrapolation_only(e, beta)
        preds[name] = e
    for name, nn_ in preds.items():
        sv = S.new_solver(case)
        sv.set_schedule(sched, tz)
        sv.set_update_chunk(tzq)
        R = S.Runner(sv, nn_, k=k, M=M)
        cross, secs, track, snap = S.time_to_domain(sv, R.advance, target, every, max_steps, snap_at=T)
        qe = float(np.linalg.norm(snap - q_plain) / np.linalg.norm(q_plain)) if snap is not None else None
        res[name] = {"steps_to_target": cross, "seconds": secs,
                     "speedup": (t_plain / secs) if (cross is not None and T is not None) else None,
                     "q_error_at_plain_crossing": qe,
                     "steps_per_second": (cross / secs) if cross is not None and secs > 0 else None,
                     "cycles": R.attempted, "fallbacks": R.fallbacks,
                     "plain_cycles": R.plain,
                     "residual_median": float(np.median(R.residuals)) if R.residuals else None,
                     "planes_every_read": [b for _, b in track]}
        log(f"bench: growth {name}: crossing {cross} steps, {secs:.3f} s, Q error {qe}")
        del sv
    for o in preds.values():
        o.close()
    # best predictor: the fastest to the target among those whose Q error at
    # the plain run's crossing stays within twice the per-cycle residual
    # threshold (the unchecked jumps of a cycle add their errors to the state)
    q_bar = 2 * S.THRESHOLD
    ok = {k_: v for k_, v in res.items() if k_ != "plain" and v["speedup"] is not None
          and v["q_error_at_plain_crossing"] is not None and v["q_error_at_plain_crossing"] <= q_bar}
    best = max(ok, key=lambda k_: ok[k_]["speedup"]) if ok else None
    net_r = res["network"]
    # a learned gain needs the network ahead of both extrapolations on the
    # driver's rate (simulated steps per second) and at the crossing, with its
    # Q error within the bar: a lead that only comes from crossing one
    # read-out earlier is not counted
    ext = [res[e] for e in ("linear_extrapolation", "quadratic_extrapolation") if e in ok]
    learned = ("network" in ok and bool(ext)
               and all(net_r["steps_per_second"] > e["steps_per_second"] for e in ext)
               and all(net_r["steps_to_target"] <= e["steps_to_target"] for e in ext))
    return {
        "workload": f"{n}^3 growing box (O2 slab z < 32 in an x-helix), kappa {kappa}, tau {tau_ldg}, FP32; "
                    f"time until the blue-phase domain reaches {target} planes (from {start} at the first "
                    f"read-out), read every {every} steps; k = {k}, M = {M}, threshold {S.THRESHOLD:g}, "
                    f"refresh {S.REFRESH:g}",
        "target_planes": target,
        "q_error_bar": q_bar,
        **res,
        "best_predictor": best,
        "learned_gain": learned,
        "increment_error_heldout": heldout,
        "training": {"pairs": n_train, "heldout_pairs": pairs_per_run, "iters": iters, "lr": lr,
                     "data_seconds": t_data, "train_seconds": tl.seconds,
                     "final_loss": tl.losses[-1][1] if tl.losses else None},
        "network_speedup_with_training": (t_plain / (net_r["seconds"] + t_data + tl.seconds))
        if net_r["speedup"] else None,
    }


def run_sizes(sizes=(64, 96, 128, 192, 256, 384, 512), site_updates=2.0e9):
    """The autotuned step on the O2 workload at several lattice sizes, FP32 and
    FP64: schedule picked, MLUPS over about `site_updates` site updates, and
    the kernels' times per launch.  Up to 128^3 the fields that the Q-side
    kernels read (Q, u, the stress) fit in the 256 MB last-level cache
    between kernels; beyond, they come from HBM."""
    import torch

    from paper_0901_3293_amd import hlb
    from paper_0901_3293_amd import inputs as I

    rows = []
    for n in sizes:
        p, Q, u, rho = I.bpii_case(n=n)
        for prec in ("fp32", "fp64"):
            s = hlb.Solver((n, n, n), prec)
            s.set_params(p)
            s.set_fields(Q, u, rho)
            sched, tz, _ = s.autotune(20)
            steps = max(20, int(site_updates / n ** 3))
            s.step(5)
            torch.cuda.synchronize()
            ev0 = torch.cuda.Event(enable_timing=True)
            ev1 = torch.cuda.Event(enable_timing=True)
            ev0.record(s.stream)
            s.step(steps)
            ev1.record(s.stream)
            torch.cuda.synchronize()
            ms = ev0.elapsed_time(ev1) / steps
            km = s.step_timed(5)
            rows.append({"n": n, "precision": prec,
                         "schedule": {"name": sched, "tz": tz, "tz_update": s.update_chunk()}, "steps": steps,
                         "ms_per_step": ms, "mlups": n ** 3 / ms / 1e3,
                         "kernel_us_per_launch": {k: v / 5 * 1e3 for k, v in km.items() if v > 0}})
            log(f"bench: size {n}^3 {prec}: {sched} tz {tz}, {rows[-1]['mlups']:.0f} MLUPS")
            s.close()
            del s
            torch.cuda.empty_cache()
        del Q, u, rho
    return {"workload": "blue-phase O2 lattice n^3 (cells of 32), autotuned schedule", "rows": rows}


def run_slab(steps=20000, every=100, kappas=(0.5, 0.8, 1.0), prec="fp32"):
    """The domain-growth slab (64 x 64 x 256, O2 seed for z < 32 inside an
    x-helix, tau_LdG = 0) for each chirality: `steps` steps with the
    plane-averaged free energy f(z) and the disclination sites per plane
    (order analysis, q < 0.19) read every `every` steps; the blue-phase
    domain is the set of planes that carry disclination sites, its walls the
    boundaries of that set."""
    import numpy as np

    from paper_0901_3293_amd import hlb
    from paper_0901_3293_amd import inputs as I
    from paper_0901_3293_amd import surrogate as S

    out = {}
    for kappa in kappas:
        p, Q, u, rho = I.slab_case(nx=64, ny=64, nz=256, cell=32, seed_depth=32, kappa=kappa)
        s = hlb.Solver((64, 64, 256), prec)
        s.set_params(p)
        s.set_fields(Q, u, rho)
        s.autotune(10)
        track = []
        t0 = time.perf_counter()
        for t in range(0, steps + 1, every):
            if t:
                s.step(every)
            fz = S.domain_profile(s)
            per_z = s.order(threshold=0.19, fields=False)["per_z"]
            mask, walls = S.defect_walls(per_z)
            f_bp = float(np.median(fz[mask])) if mask.any() else None
            f_ch = float(np.median(fz[~mask])) if (~mask).any() else None
            track.append({"step": t, "bp_planes": int(mask.sum()), "walls": walls,
                          "defect_sites": int(np.sum(per_z)), "f_bp": f_bp, "f_cholesteric": f_ch})
        el = time.perf_counter() - t0
        keep = (0, 100, 500, 1000, 2000, 5000, 10000, 15000, 20000)
        out[str(kappa)] = {"seconds": el, "mlups_with_readouts": 64 * 64 * 256 * steps / el / 1e6,
                           "track": [r for r in track if r["step"] in keep],
                           "bp_planes_every_1000": [r["bp_planes"] for r in track if r["step"] % 1000 == 0]}
        log(f"bench: slab kappa {kappa}: blue-phase planes {track[0]['bp_planes']} -> {track[-1]['bp_planes']}, "
            f"walls {track[-1]['walls']}")
        s.close()
    return {"workload": f"64x64x256 domain-growth slab (O2 seed z < 32 in an x-helix, tau_LdG = 0), {prec}, "
                        f"{steps} steps, f(z) and disclinations per plane every {every}", "kappa": out}


def run_network(n=96, predicts=20, train_steps=10):
    """The surrogate network alone on an n^3 lattice with seeded random
    inputs: `predicts` forward applications, then `train_steps` training
    steps (forward, backward, Adam).  For kernel profiles."""
    import numpy as np
    import torch

    from paper_0901_3293_amd import hlb
    from paper_0901_3293_amd import inputs as I

    N = n ** 3
    net = hlb.Net((n, n, n))
    net.set_params(I.cnn_params(seed=0))
    norm = np.zeros(net.n_norm, dtype=np.float32)
    norm[net.n_in:2 * net.n_in] = 1.0
    norm[2 * net.n_in + 5:2 * net.n_in + 10] = 1.0
    net.set_norm(norm)
    g = torch.Generator(device="cuda").manual_seed(0)
    x = torch.randn((net.n_in, N), device="cuda", generator=g)
    y = torch.randn((5, N), device="cuda", generator=g) * 0.1
    out = torch.empty((5, N), device="cuda")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    net.predict(x, out)
    e0.record(net.stream)
    for _ in range(predicts):
        net.predict(x, out)
    e1.record(net.stream)
    torch.cuda.synchronize()
    ms_pred = e0.elapsed_time(e1) / predicts
    net.train_step(x, y, 1e-5, want_loss=False)
    e0.record(net.stream)
    for _ in range(train_steps):
        net.train_step(x, y, 1e-5, want_loss=False)
    e1.record(net.stream)
    torch.cuda.synchronize()
    ms_train = e0.elapsed_time(e1) / train_steps
    net.close()
    return {"lattice": n, "predict_ms": ms_pred, "train_step_ms": ms_train}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(n, budget_s=15.0, budget_one_s=10.0):
    """The FP64 oracle (test infrastructure) on the host: steps of the same
    128^3 workload until the time budget is spent (at least one step), with
    the oracle's default OpenMP thread count, then with one thread."""
    import oracle
    from paper_0901_3293_amd import inputs as I

    p, Q, u, rho = I.bpii_case(n=n)
    st = oracle.State(oracle.params(**p.as_dict()), Q, u, rho)

    def timed(budget):
        st.step(1)  # warm caches and the OpenMP pool
        done, t0 = 0, time.perf_counter()
        while True:
            st.step(1)
            done += 1
            el = time.perf_counter() - t0
            if el >= budget:
                return done, el

    cores = oracle.max_threads()
    done, el = timed(budget_s)
    oracle.set_threads(1)
    done1, el1 = timed(budget_one_s)
    oracle.set_threads(cores)
    return {"value": n ** 3 * done / el / 1e6, "unit": "MLUPS", "cores": cores, "kind": "oracle",
            "sample": f"{done} FP64 oracle steps of the {n}^3 workload ({el:.1f} s)",
            "one_thread": {"value": n ** 3 * done1 / el1 / 1e6, "unit": "MLUPS",
                           "sample": f"{done1} steps ({el1:.1f} s)"},
            "host": {"cpu_model": cpu_model(), "nproc": os.cpu_count()}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--prof-steps", type=int, default=20)
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--only", choices=["fp32", "fp64", "batched", "surrogate", "surrogate-mixed", "network", "order",
                                       "slab", "sizes"], default=None,
                    help="run one leg only (profiling runs)")
    ap.add_argument("--coupling", choices=["force", "split"], default="force",
                    help="fluid coupling of the --only fp32/fp64 profiling legs")
    ap.add_argument("--no-split", action="store_true", help="skip the FP32 split-coupling and D3Q15 legs")
    ap.add_argument("--lb-model", choices=["d3q19", "d3q15"], default="d3q19",
                    help="LB scheme of the --only fp32/fp64 profiling legs (d3q15 implies --coupling split)")
    ap.add_argument("--schedule", choices=["auto", "sites", "tiled", "mixed", "fused", "fused-tiled"],
                    default="auto", help="step schedule (auto: the library's autotuner picks)")
    ap.add_argument("--tz", type=int, default=0, help="planes per tile column for a fixed schedule with tiles")
    ap.add_argument("--tz-update", type=int, default=0,
                    help="planes per tile column of the tiled Q update, if other than --tz")
    ap.add_argument("--batch-steps", type=int, default=1000,
                    help="steps of the 96-box batched FP32 run (0: skip)")
    ap.add_argument("--batch-graph-steps", type=int, default=50, help="steps per batched graph replay")
    ap.add_argument("--batch-chunk", type=int, default=0,
                    help="fixed chunk for every box size instead of the autotuner (profiling runs)")
    ap.add_argument("--batch-launch", choices=["persistent", "phases"], default=None,
                    help="batched launch form (default: the autotuner's pick; with --batch-chunk: the library default, phases)")
    ap.add_argument("--batch-group", type=int, default=0,
                    help="cache-group budget in sites (persistent form: group_sites / 8 per XCD group; 0: the autotuner's)")
    ap.add_argument("--batch-device-fences", action="store_true",
                    help="batched run with the fixed work mapping and device-scope barrier fences")
    ap.add_argument("--slab-steps", type=int, default=20000,
                    help="steps of the 64x64x256 domain-growth slab per chirality (0: skip)")
    ap.add_argument("--surrogate-steps", type=int, default=20000,
                    help="steps of the 96^3 surrogate-vs-plain run of --only surrogate-mixed")
    ap.add_argument("--no-surrogate", action="store_true", help="skip the surrogate time-to-domain-size leg")
    ap.add_argument("--growth-target", type=int, default=44,
                    help="blue-phase planes the growing 96^3 box must reach (surrogate leg)")
    ap.add_argument("--growth-every", type=int, default=128,
                    help="steps between domain read-outs (a multiple of k M)")
    ap.add_argument("--growth-max-steps", type=int, default=30720, help="steps before a run gives up")
    ap.add_argument("--growth-kappa", type=float, default=1.0, help="chirality of the growing box")
    ap.add_argument("--surrogate-k", type=int, default=32, help="solver steps replaced by one network jump")
    ap.add_argument("--surrogate-m", type=int, default=4, help="jumps per checked surrogate cycle")
    ap.add_argument("--surrogate-iters", type=int, default=3000, help="training iterations of the surrogate")
    ap.add_argument("--surrogate-train", choices=["mixed", "growth"], default="mixed",
                    help="training pairs: O2 and domain-growth runs, or domain-growth runs only")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 512 MiB device copy (calibrates HBM byte counters)")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py measures one GPU only (the step is single-device; --gpus {a.gpus} is not "
              "supported)", file=sys.stderr)
        sys.exit(2)
    import torch

    assert torch.cuda.is_available(), "bench needs a HIP device"
    if a.copy_probe:
        src = torch.empty(512 << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("bench: copy probe 512 MiB x3 done")
        del src, dst
    if a.only in ("batched", "surrogate", "surrogate-mixed", "network", "order", "slab", "sizes"):
        if a.only == "order":
            out = run_order(a.n)
        elif a.only == "sizes":
            out = run_sizes()
        elif a.only == "slab":
            out = run_slab()
        elif a.only == "batched":
            out = run_batched(a.batch_steps, a.batch_graph_steps, a.batch_chunk, not a.batch_device_fences,
                              a.batch_launch, a.batch_group)
        elif a.only == "network":
            out = run_network()
        elif a.only == "surrogate":
            out = run_surrogate_growth(kappa=a.growth_kappa, target=a.growth_target, every=a.growth_every,
                                       max_steps=a.growth_max_steps, k=a.surrogate_k, M=a.surrogate_m,
                                       iters=a.surrogate_iters)
        else:
            out = run_surrogate(steps=a.surrogate_steps, k=a.surrogate_k, M=a.surrogate_m, iters=a.surrogate_iters,
                                train_set=a.surrogate_train)
        print(json.dumps({"profiling_run": a.only, **out}), flush=True)
        return
    res = {}
    forms = (a.only,) if a.only else ("fp32", "fp64")
    for prec in forms:
        log(f"bench: {prec} {a.n}^3, warmup {a.warmup}, steps {a.steps}")
        if a.only and a.lb_model == "d3q15":
            a.coupling = "split"
        res[prec] = run_form(prec, a.n, a.steps, a.warmup, a.prof_steps, a.schedule, a.tz,
                             a.coupling if a.only else "force", a.lb_model if a.only else "d3q19", a.tz_update)
        log(f"bench: {prec} {res[prec]['mlups']:.1f} MLUPS, kernels {res[prec]['kernel_ms_per_launch']}")
    split = d3q15 = None
    if not a.only and not a.no_split:
        log(f"bench: fp32 {a.n}^3 split coupling")
        r = run_form("fp32", a.n, a.steps, a.warmup, a.prof_steps, "auto", 0, "split")
        split = {k: r[k] for k in ("mlups", "ms_per_step", "schedule", "kernel_ms_per_launch", "roofline",
                                   "step_roofline")}
        log(f"bench: split {split['mlups']:.1f} MLUPS")
        log(f"bench: fp32 {a.n}^3 D3Q15 predictor-corrector LB, split coupling")
        r = run_form("fp32", a.n, a.steps, a.warmup, a.prof_steps, "auto", 0, "split", "d3q15")
        d3q15 = {k: r[k] for k in ("mlups", "ms_per_step", "schedule", "kernel_ms_per_launch", "roofline",
                                   "step_roofline")}
        log(f"bench: d3q15 {d3q15['mlups']:.1f} MLUPS")
    order = None
    if not a.only:
        log(f"bench: order analysis {a.n}^3")
        order = run_order(a.n)
    batched = None
    if a.batch_steps > 0 and not a.only:
        log(f"bench: batched 96 boxes fp32, {a.batch_steps} steps")
        batched = run_batched(a.batch_steps)
        log(f"bench: batched {batched['mlups']:.1f} MLUPS aggregate")
    growth = None
    if a.slab_steps > 0 and not a.only:
        log(f"bench: domain-growth slab 64x64x256, {a.slab_steps} steps, three chiralities")
        sl = run_slab(steps=a.slab_steps)
        growth = {"workload": sl["workload"],
                  "blue_phase_planes_every_1000": {k: v["bp_planes_every_1000"] for k, v in sl["kappa"].items()},
                  "final": {k: v["track"][-1] for k, v in sl["kappa"].items()},
                  "mlups_with_readouts": {k: v["mlups_with_readouts"] for k, v in sl["kappa"].items()}}
    sur = None
    if not a.no_surrogate and not a.only:
        log(f"bench: surrogate, time to {a.growth_target} blue-phase planes on the growing 96^3 box, "
            f"k {a.surrogate_k}, M {a.surrogate_m}")
        sur = run_surrogate_growth(kappa=a.growth_kappa, target=a.growth_target, every=a.growth_every,
                                   max_steps=a.growth_max_steps, k=a.surrogate_k, M=a.surrogate_m,
                                   iters=a.surrogate_iters)
        log(f"bench: surrogate best predictor {sur['best_predictor']}")
    cpu = None
    if not a.no_cpu:
        log("bench: cpu baseline (oracle)")
        cpu = cpu_baseline(a.n, a.cpu_budget)
    if a.only:
        print(json.dumps({"profiling_run": a.only, **res[a.only]}), flush=True)
        return
    r32, r64 = res["fp32"], res["fp64"]
    line = {
        "metric": "coupled-step MLUPS (FP32 form; FP64 alongside) + % HBM roofline",
        "value": r32["mlups"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": r32["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"blue-phase O2 lattice {a.n}^3 periodic (4^3 cells of 32), D3Q19 "
                               "hybrid LB, kappa=0.7 tau=-0.5",
                   "lattice": [a.n, a.n, a.n], "sites": a.n ** 3, "parallelism": "single GPU"},
        "roofline": r32["roofline"],
        "step_roofline": r32["step_roofline"],
        "kernel_ms_per_launch": r32["kernel_ms_per_launch"],
        "schedule": r32["schedule"],
        "fp64": {"value": r64["mlups"], "unit": "MLUPS", "dtype": "f64", "ms_per_step": r64["ms_per_step"],
                 "schedule": r64["schedule"],
                 "roofline": r64["roofline"], "step_roofline": r64["step_roofline"],
                 "kernel_ms_per_launch": r64["kernel_ms_per_launch"]},
        "split_coupling_fp32": split,
        "d3q15_predictor_corrector_fp32": d3q15,
        "order": order,
        "batched": batched,
        "domain_growth": growth,
        "surrogate": sur,
        "checks": {"fp32": r32["checks"], "fp64": r64["checks"]},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
