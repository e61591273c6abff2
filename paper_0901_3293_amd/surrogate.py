"""Training and use of the convolutional surrogate of the slow Q dynamics.

The surrogate replaces k solver steps by one application of a small 3D CNN
that maps the current state (Q, u) and the recent history of Q (the last
k-step increment d1 and its change s2) to the increment of Q over the next k
steps, as a correction to the extrapolation d1 + beta s2.  The plain step
checks its error: every M-th jump is repeated with k plain steps
and the whole cycle is redone with plain steps when the relative residual
reaches a threshold (``hlb_surrogate_advance``).

This module only schedules work: solver runs that generate training pairs
(``hlbnn_make_pair``), the standardisation (``hlbnn_fit_norm``), the training
loop (``hlbnn_train_step``: forward, loss, backward, Adam) and the
surrogate-with-fallback run.  Every arithmetic step of training and inference
runs in the library's kernels; torch provides device memory only, plus the
error norms used to report results.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import hlb, inputs

K_JUMP = 8            # solver steps replaced by one network application
THRESHOLD = 1e-3      # relative residual from which a cycle falls back
REFRESH = 0.1         # fraction of THRESHOLD from which an accepted cycle is followed by a plain one
N_IN = 18             # network inputs: Q (5), u (3), d1 (5), s2 (5)


# --------------------------------------------------------------------------
# Workloads
# --------------------------------------------------------------------------

def o2_run(n=96, cell=32, kappa=0.7, tau_ldg=-0.5, noise_amp=1e-3, seed=0):
    """A double-twist (O2) lattice of side-`cell` unit cells on an n^3 box with
    seeded uniform noise on Q: the source of training trajectories."""
    p, Q, u, rho = inputs.bpii_case(n=n, cell=cell, kappa=kappa, tau_ldg=tau_ldg)
    Q = Q + inputs.noise((n, n, n), noise_amp, seed)
    return p, Q, u, rho


def growth_run(n=96, cell=32, seed_depth=32, kappa=0.7, tau_ldg=-0.5, noise_amp=0.0, seed=0):
    """Domain-growth box: an O2 slab z < seed_depth inside a cholesteric helix
    with its axis along x."""
    p, Q, u, rho = inputs.slab_case(nx=n, ny=n, nz=n, cell=cell, seed_depth=seed_depth, kappa=kappa,
                                    tau_ldg=tau_ldg)
    if noise_amp:
        Q = Q + inputs.noise((n, n, n), noise_amp, seed)
    return p, Q, u, rho


def new_solver(case, precision="fp32", stream=None):
    p, Q, u, rho = case
    nz, ny, nx = Q.shape[1:]
    s = hlb.Solver((nx, ny, nz), precision, stream=stream)
    s.set_params(p)
    s.set_fields(Q, u, rho)
    return s


# --------------------------------------------------------------------------
# Training data
# --------------------------------------------------------------------------

@dataclass
class PairSet:
    """Training pairs on the device: X [P, 18, N] raw inputs (Q, u, d1, s2),
    Y [P, 5, N] raw increments of Q over the next k steps, and the solver
    time and source run of each pair."""
    X: torch.Tensor
    Y: torch.Tensor
    times: list = field(default_factory=list)
    sources: list = field(default_factory=list)

    def __len__(self):
        return self.X.shape[0]


def allocate_pairs(n_pairs, N, device="cuda"):
    return PairSet(torch.empty((n_pairs, N_IN, N), dtype=torch.float32, device=device),
                   torch.empty((n_pairs, 5, N), dtype=torch.float32, device=device))


def record_pairs(net, solver, pairs, first, count, spacing, k=K_JUMP, burn_in=0, tag=""):
    """Run `solver` and store `count` pairs into slots first..first+count-1:
    after `burn_in` steps, one pair every `spacing` steps (each pair takes
    a 2k-step history warm-up and k steps)."""
    if spacing < 3 * k:
        raise ValueError("spacing must be at least 3k")
    t = 0
    if burn_in:
        solver.step(burn_in)
        t = burn_in
    for j in range(count):
        if j:
            solver.step(spacing - 3 * k)
            t += spacing - 3 * k
        net.make_pair(solver, k, pairs.X[first + j], pairs.Y[first + j])
        pairs.times.append(t + 2 * k)
        pairs.sources.append(tag)
        t += 3 * k
    return t


def fit_norm(net, pairs, beta, index=None):
    """Per-channel standardisation of inputs and targets (the correction to
    d1 + beta s2) from the pairs (all, or the contiguous slots `index`)."""
    if index is None:
        return net.fit_norm(pairs.X, pairs.Y, beta)
    lo, hi = min(index), max(index) + 1
    assert list(index) == list(range(lo, hi)), "fit_norm takes a contiguous run of pairs"
    return net.fit_norm(pairs.X[lo:hi], pairs.Y[lo:hi], beta)


# --------------------------------------------------------------------------
# Training
# --------------------------------------------------------------------------

@dataclass
class TrainLog:
    losses: list
    seconds: float
    steps: int


def lr_at(it, total, lr0, lr_min_frac=0.05, warmup=20):
    """Linear warm-up, then cosine decay to lr_min_frac * lr0."""
    if it < warmup:
        return lr0 * (it + 1) / warmup
    x = (it - warmup) / max(1, total - warmup)
    return lr0 * (lr_min_frac + (1 - lr_min_frac) * 0.5 * (1 + math.cos(math.pi * min(1.0, x))))


def train(net, pairs, iters, lr=2e-3, seed=0, index=None, log_every=50, progress=None):
    """Adam on single-field minibatches drawn in seeded random order (one
    epoch = one pass over `index`, default all pairs)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    idx = np.arange(len(pairs)) if index is None else np.asarray(index)
    order = []
    losses = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for it in range(iters):
        if not order:
            order = list(rng.permutation(idx))
        j = int(order.pop())
        want = (it % log_every == 0) or it == iters - 1
        loss = net.train_step(pairs.X[j], pairs.Y[j], lr_at(it, iters, lr), want_loss=want)
        if want:
            losses.append((it, loss))
            if progress:
                progress(it, loss)
    torch.cuda.synchronize()
    return TrainLog(losses, time.perf_counter() - t0, iters)


def evaluate(net, pairs, index):
    """Relative error ||dQ_pred - dQ|| / ||dQ|| of the next k-step increment
    per pair for the network and for the extrapolations it corrects: zero
    increment (1 by definition), linear (d1) and quadratic (d1 + s2); and the
    network's error relative to ||Q(t+k)|| (the residual the driver tests)."""
    out = {"net": [], "linear": [], "quadratic": [], "net_resid": []}
    for j in index:
        x, y = pairs.X[j].double(), pairs.Y[j].double()
        d1, s2 = x[8:13], x[13:18]
        pred = net.predict(pairs.X[j]).reshape(5, -1).double()
        ny = torch.linalg.vector_norm(y).item()
        qn = torch.linalg.vector_norm(x[:5] + y).item()
        err = lambda p: torch.linalg.vector_norm(p - y).item()
        out["net"].append(err(pred) / ny)
        out["linear"].append(err(d1) / ny)
        out["quadratic"].append(err(d1 + s2) / ny)
        out["net_resid"].append(err(pred) / qn)
    return {k: np.array(v) for k, v in out.items()}


# --------------------------------------------------------------------------
# Surrogate run
# --------------------------------------------------------------------------

@dataclass
class RunStats:
    steps: int
    cycles: int          # surrogate cycles attempted
    fallbacks: int       # of which rolled back and redone with plain steps
    plain_cycles: int    # cycles taken with plain steps while cooling down
    residuals: list
    seconds: float
    fallback_steps: list = field(default_factory=list)  # solver step at which each fallback cycle began


class Runner:
    """Cycles of M*k solver steps on one solver with the surrogate policy.

    A cycle is a surrogate cycle (M network jumps, the last one checked
    against k plain steps, rolled back to plain steps when its residual
    reaches `threshold`) unless the runner is cooling down: after a fallback
    the next c cycles are plain (c = 1, 2, 4, ... up to cooldown_max on
    consecutive fallbacks, reset by an accepted cycle), so a fast transient is
    not paid for twice.  An accepted cycle whose residual reaches
    refresh * threshold is followed by one plain cycle (refresh=None turns
    this off): the errors of the unchecked jumps accumulate in the state, and
    a plain cycle taken before the check fails costs less than a rolled-back
    one.  A plain cycle leaves a valid history behind (its last 2k steps are
    the network's warm-up)."""

    def __init__(self, solver, net, k=K_JUMP, M=8, threshold=THRESHOLD, cooldown_max=64, refresh=REFRESH):
        self.solver, self.net, self.k, self.M = solver, net, k, M
        self.threshold, self.cooldown_max, self.refresh = threshold, cooldown_max, refresh
        self.cyc = k * M
        self.wait = 0
        self.penalty = 1
        self.steps = 0
        self.attempted = self.fallbacks = self.plain = 0
        self.residuals = []
        self.fallback_steps = []

    def plain_cycle(self):
        self.solver.step(self.cyc - 2 * self.k)
        self.net.warmup(self.solver, self.k)
        self.steps += self.cyc

    def cycle(self):
        if self.wait > 0:
            self.plain_cycle()
            self.wait -= 1
            self.plain += 1
            return
        f, r = hlb.surrogate_advance(self.solver, self.net, k=self.k, M=self.M, threshold=self.threshold)
        self.attempted += 1
        self.residuals.append(r)
        if f:
            self.fallbacks += 1
            self.fallback_steps.append(self.steps)
            self.wait = self.penalty
            self.penalty = min(2 * self.penalty, self.cooldown_max)
        else:
            self.penalty = 1
            if self.refresh is not None and r >= self.refresh * self.threshold:
                self.wait = 1
        self.steps += self.cyc

    def advance(self, nsteps):
        """nsteps (a multiple of the cycle length) more steps; the first cycle
        of a run is a plain one, which records the network's history."""
        if nsteps % self.cyc:
            raise ValueError(f"advance({nsteps}) is not a whole number of {self.cyc}-step cycles")
        for _ in range(nsteps // self.cyc):
            if self.steps == 0:
                self.plain_cycle()
            else:
                self.cycle()

    def stats(self, seconds):
        return RunStats(self.steps, self.attempted, self.fallbacks, self.plain, self.residuals, seconds,
                        self.fallback_steps)


def run(solver, net, steps, k=K_JUMP, M=8, threshold=THRESHOLD, cooldown_max=64, refresh=REFRESH):
    """Advance `solver` by `steps` solver steps: a 2k-step history warm-up,
    then cycles of M*k steps (Runner) while a whole cycle fits, plain steps
    for the rest."""
    R = Runner(solver, net, k, M, threshold, cooldown_max, refresh)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    net.warmup(solver, k)
    R.steps = 2 * k
    n_cyc = (steps - 2 * k) // R.cyc
    for _ in range(n_cyc):
        R.cycle()
    rest = steps - R.steps
    if rest:
        solver.step(rest)
        R.steps += rest
    torch.cuda.synchronize()
    st = R.stats(time.perf_counter() - t0)
    st.fallback_steps = list(R.fallback_steps)
    return st


def blue_phase_planes(solver, threshold=0.19):
    """Planes of the blue-phase domain: z-planes carrying disclination sites
    (local order below the threshold; the cholesteric carries none)."""
    return int((solver.order(threshold=threshold, fields=False)["per_z"] > 0).sum())


def time_to_domain(solver, advance, target, every, max_steps, snap_at=None):
    """Advance `solver` with `advance(n)` in chunks of `every` steps, reading
    the blue-phase planes after each chunk, until they reach `target` or
    `max_steps` steps have run (and at least `snap_at` steps, where Q is
    copied to the host).  Only the stepping is timed (device synchronised
    around each chunk).  Returns (steps at the crossing or None, seconds
    to the crossing, track [(step, planes)], Q at snap_at or None)."""
    t, secs, track, snap, cross, cross_s = 0, 0.0, [], None, None, None
    while t < max_steps and (cross is None or (snap_at is not None and t < snap_at)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        advance(every)
        torch.cuda.synchronize()
        secs += time.perf_counter() - t0
        t += every
        bp = blue_phase_planes(solver)
        track.append((t, bp))
        if cross is None and bp >= target:
            cross, cross_s = t, secs
        if snap_at is not None and t == snap_at:
            snap = solver.fields()[0]
    return cross, cross_s, track, snap


def plain_run(solver, steps):
    """The plain FP32 form over the same steps, timed the same way."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    solver.step(steps)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def extrapolation_only(net, beta):
    """Turn `net` into the method without the network: every jump is the
    extrapolation d1 + beta s2 (all weights zero, target mean zero)."""
    net.set_params(np.zeros(net.n_params, dtype=np.float32))
    norm = np.zeros(net.n_norm, dtype=np.float32)
    norm[N_IN:2 * N_IN] = 1.0
    norm[2 * N_IN + 5:2 * N_IN + 10] = 1.0
    norm[2 * N_IN + 10] = beta
    net.set_norm(norm)


def q_error(a, b):
    """||Q_a - Q_b|| / ||Q_b|| over all sites and the five stored components."""
    Qa, Qb = a.fields()[0], b.fields()[0]
    return float(np.linalg.norm(Qa - Qb) / np.linalg.norm(Qb))


def domain_profile(solver):
    """Plane-averaged free-energy density f(z)."""
    nx, ny, _ = solver.shape
    return solver.fz() / (nx * ny)


def domain_size(fz):
    """Planes of the higher free-energy phase: the number of z-planes whose
    plane-averaged f lies above the midpoint of the profile's extremes."""
    fz = np.asarray(fz)
    return int((fz > 0.5 * (fz.max() + fz.min())).sum())


def defect_walls(per_z):
    """Blue-phase planes and domain walls of a periodic box from the
    disclination sites per z-plane (order analysis): a plane carrying
    disclination sites belongs to the blue-phase domain (the cholesteric
    carries none); a wall sits between two neighbouring planes of different
    kind, at z + 1/2.  Returns (mask of blue-phase planes, wall positions)."""
    mask = np.asarray(per_z) > 0
    nz = len(mask)
    walls = [z + 0.5 for z in range(nz) if mask[z] != mask[(z + 1) % nz]]
    return mask, walls


# Multiply-adds per site of one network application (3x3x3 taps, real channels).
MACS_PER_SITE = 27 * (N_IN * 32 + 32 * 32 + 32 * 32 + 32 * 5)
