"""The item-claiming rule of the persistent batched kernel, modelled on the host.

Within a phase the `per` workgroups of a group take items from the group's
counter one claim at a time: a claim v names item v - base if that is below
the phase's item count n, and a workgroup stops after its first claim past
the items.  The kernel then starts the next phase at base + n + per, without
reading the counter.  That is only right if every phase advances the counter
by exactly n + per whatever the interleaving of the claims; the model below
runs the rule with random interleavings (a workgroup's next claim is issued
while it works on the current item, as thread 0 does in the kernel) and
checks that, and that every item is processed exactly once."""
import random

import pytest


def run_phase(counter, base, n, per, rng):
    """One phase: returns (counter after, items processed in order)."""
    done = []
    # each workgroup: its first claim, then one claim per item it works on
    pending = {w: None for w in range(per)}
    active = set(range(per))
    while active:
        w = rng.choice(sorted(active))
        v = counter
        counter += 1
        item = v - base if v - base < n else -1
        if pending[w] is not None:
            done.append(pending[w])  # finish the current item, keep the claim as the next one
        if item < 0:
            active.discard(w)
            pending[w] = None
        else:
            pending[w] = item
    return counter, done


@pytest.mark.parametrize("seed", range(20))
def test_claims_cover_every_item_once_and_advance_by_n_plus_per(seed):
    rng = random.Random(seed)
    counter, base = 0, 0
    for _ in range(30):  # phases of several cache groups
        n = rng.randint(0, 300)
        per = rng.randint(1, 64)
        counter, done = run_phase(counter, base, n, per, rng)
        assert sorted(done) == list(range(n))
        base += n + per
        assert counter == base


def test_a_workgroup_with_no_item_makes_exactly_one_claim():
    rng = random.Random(1)
    counter, done = run_phase(0, 0, 0, 8, rng)
    assert done == [] and counter == 8
