"""Host logic of the surrogate run (`surrogate.run`): step accounting, the
cool-down after a fallback and the refresh after an accepted cycle with a
large residual; and the domain-wall finder of the growth runs.  The solver, the network and the checked cycle are stand-ins
that count steps and return scripted residuals; nothing touches a GPU."""
import pytest

from paper_0901_3293_amd import surrogate as S


class Clock:
    """Solver steps taken, and the kind of each cycle in order."""

    def __init__(self):
        self.steps = 0
        self.log = []


class FakeSolver:
    def __init__(self, clock):
        self.c = clock

    def step(self, n):
        self.c.steps += n


class FakeNet:
    def __init__(self, clock):
        self.c = clock

    def warmup(self, solver, k):
        self.c.steps += 2 * k  # two k-step increments of history


def run(monkeypatch, script, steps, k=4, M=3, **kw):
    """Run the policy with surrogate cycles returning (fell_back, residual)
    from `script` in order; returns the stats and the clock."""
    clock = Clock()
    it = iter(script)

    def advance(solver, net, k, M, threshold):
        f, r = next(it)
        clock.steps += M * k
        clock.log.append("F" if f else "S")
        return f, r

    monkeypatch.setattr(S.hlb, "surrogate_advance", advance)
    monkeypatch.setattr(S.torch.cuda, "synchronize", lambda: None)
    solver, net = FakeSolver(clock), FakeNet(clock)
    orig_step = solver.step

    def step(n):
        if n == M * k - 2 * k:
            clock.log.append("P")
        orig_step(n)

    solver.step = step
    st = S.run(solver, net, steps, k=k, M=M, **kw)
    return st, clock


@pytest.mark.parametrize("steps", [8, 20, 8 + 12 * 5, 8 + 12 * 5 + 7])
def test_steps_add_up(monkeypatch, steps):
    st, clock = run(monkeypatch, [(False, 1e-5)] * 100, steps)
    assert clock.steps == steps
    assert st.cycles == (steps - 8) // 12 and st.fallbacks == 0 and st.plain_cycles == 0


def test_cooldown_doubles_and_resets(monkeypatch):
    """Fallback, fallback, accept, fallback: plain cycles 1, then 2, then none,
    then 1 again (the penalty was reset by the accepted cycle)."""
    script = [(True, 2e-3), (True, 2e-3), (False, 1e-5), (True, 2e-3), (False, 1e-5), (False, 1e-5)]
    st, clock = run(monkeypatch, script, 8 + 12 * 10, refresh=None)
    assert "".join(clock.log) == "FPFPPSFPSS"
    assert st.fallbacks == 3 and st.plain_cycles == 4 and st.cycles == 6
    assert clock.steps == 8 + 12 * 10
    assert st.fallback_steps == [8, 8 + 2 * 12, 8 + 6 * 12]


def test_cooldown_is_capped(monkeypatch):
    st, clock = run(monkeypatch, [(True, 1.0)] * 10, 8 + 12 * (1 + 1 + 2 + 2 + 1 + 2 + 1), cooldown_max=2,
                    refresh=None)
    assert "".join(clock.log) == "FPFPPFPPFP"


def test_refresh_after_large_accepted_residual(monkeypatch):
    """An accepted cycle at or above refresh * threshold is followed by one
    plain cycle; below it, by another surrogate cycle."""
    thr = 1e-3
    script = [(False, 1e-5), (False, 1e-4), (False, 0.99e-4), (False, 5e-4), (False, 1e-6)]
    st, clock = run(monkeypatch, script, 8 + 12 * 7, threshold=thr, refresh=0.1)
    assert "".join(clock.log) == "SSPSSPS"
    assert st.plain_cycles == 2 and st.fallbacks == 0 and st.cycles == 5
    # the same residuals without the rule: no plain cycles
    st2, clock2 = run(monkeypatch, script, 8 + 12 * 5, threshold=thr, refresh=None)
    assert "".join(clock2.log) == "SSSSS" and st2.plain_cycles == 0


def test_refresh_is_the_default(monkeypatch):
    st, clock = run(monkeypatch, [(False, S.REFRESH * S.THRESHOLD), (False, 0.0)], 8 + 12 * 3)
    assert "".join(clock.log) == "SPS"


def test_defect_walls_periodic():
    """A blue-phase slab on planes 0..31 of 256 (disclination sites there,
    none elsewhere): walls between planes 31|32 and 255|0, 32 blue-phase
    planes; a box without disclinations has no walls."""
    import numpy as np

    per_z = np.zeros(256, dtype=np.int64)
    per_z[0:32] = np.arange(1, 33)
    mask, walls = S.defect_walls(per_z)
    assert mask.sum() == 32 and walls == [31.5, 255.5]
    assert S.defect_walls(np.zeros(8))[1] == []


def test_runner_advance_starts_plain_and_counts_steps(monkeypatch):
    """Runner.advance in chunks: the first cycle of a run is plain (it records
    the history), every later one follows the policy; steps add up per chunk,
    and a chunk that is not a whole number of cycles is refused."""
    clock = Clock()
    script = iter([(False, 1e-5), (True, 2e-3), (False, 1e-5), (False, 1e-5)])

    def advance(solver, net, k, M, threshold):
        f, r = next(script)
        clock.steps += M * k
        clock.log.append("F" if f else "S")
        return f, r

    monkeypatch.setattr(S.hlb, "surrogate_advance", advance)
    solver, net = FakeSolver(clock), FakeNet(clock)
    orig = solver.step

    def step(n):
        clock.log.append("P")
        orig(n)

    solver.step = step
    R = S.Runner(solver, net, k=4, M=3, refresh=None)
    R.advance(24)
    assert clock.steps == 24 and R.steps == 24 and "".join(clock.log) == "PS"
    R.advance(36)
    assert clock.steps == 60 and R.steps == 60 and "".join(clock.log) == "PSFPS"
    assert R.fallbacks == 1 and R.plain == 1 and R.attempted == 3
    with pytest.raises(ValueError):
        R.advance(13)


def test_time_to_domain_stops_at_target_and_snapshots(monkeypatch):
    """time_to_domain reads the blue-phase planes after each chunk, reports
    the first chunk at or above the target, and keeps going to the snapshot
    step when that comes later."""
    import numpy as np

    monkeypatch.setattr(S.torch.cuda, "synchronize", lambda: None)

    class GrowingSolver:
        def __init__(self):
            self.t = 0

        def step(self, n):
            self.t += n

        def order(self, threshold=0.19, fields=False):
            planes = 10 + self.t // 100  # one plane per 100 steps
            per_z = np.zeros(64, dtype=np.int64)
            per_z[:planes] = 1
            return {"per_z": per_z}

        def fields(self):
            return np.full((5, 1, 1, 1), float(self.t)), None, None

    s = GrowingSolver()
    cross, secs, track, snap = S.time_to_domain(s, s.step, target=14, every=50, max_steps=1000, snap_at=600)
    assert cross == 400 and track[7] == (400, 14) and s.t == 600 and snap[0, 0, 0, 0] == 600.0
    s2 = GrowingSolver()
    cross2, _, track2, snap2 = S.time_to_domain(s2, s2.step, target=99, every=100, max_steps=500)
    assert cross2 is None and len(track2) == 5 and snap2 is None
