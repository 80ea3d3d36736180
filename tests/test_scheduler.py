"""Adaptive keyframe selection (Eqs. (5)-(8)): the library's C++ scheduler
against the plain Python oracle, and the refill rule against hand-worked
cases of Eq. (8)."""
import math

import numpy as np

from oracle.scheduler import Scheduler
from paper_2410_00486_amd import KeyframeScheduler


def test_refill_rule_hand_worked():
    # k = 8 keyframes, d = 4 -> d_k = 2: the two largest losses get 2 iterations
    s = KeyframeScheduler(capacity=16, r0=1, d=4)
    ids = [s.add_keyframe() for _ in range(8)]
    losses = [0.5, 3.0, 1.0, 3.0, 0.1, 2.9, 0.2, 0.3]
    for i in ids:
        assert s.select([0.0]) != []          # drain the initial r0 = 1 counts
    for i, l in zip(ids, losses):
        s.report(i, l)
    assert s.remaining == [0] * 8
    s.select([0.0])                           # triggers the refill, then picks index 0
    # ties at 3.0 -> both indices 1 and 3 are in the top 2
    assert s.remaining == [0, 2, 1, 2, 1, 1, 1, 1]
    assert s.refills == 1
    # k = 3, d = 4 -> d_k = max(1, 0) = 1
    t = KeyframeScheduler(capacity=4, r0=1, d=4)
    for _ in range(3):
        t.add_keyframe()
    for _ in range(3):
        t.select([0.99])
    t.report(0, 1.0)
    t.report(1, 1.0)
    t.report(2, 0.5)
    # refill: the tie at the largest loss goes to index 0 -> r = [2, 1, 1];
    # u = 0.5 then picks position floor(1.5) = 1 of the eligible [0, 1, 2]
    assert t.select([0.5]) == [1]
    assert t.remaining == [2, 0, 1]


def test_new_keyframe_has_infinite_loss_and_r0():
    s = KeyframeScheduler(capacity=8, r0=8, d=4)
    i = s.add_keyframe()
    assert s.remaining == [8] and math.isinf(s.losses[i])


def test_library_matches_oracle_on_random_sequences():
    rng = np.random.default_rng(0)
    for trial in range(20):
        r0, d, batch = int(rng.integers(1, 9)), int(rng.integers(1, 6)), int(rng.integers(1, 5))
        lib, ref = KeyframeScheduler(capacity=256, r0=r0, d=d), Scheduler(r0=r0, d=d)
        for it in range(400):
            if rng.uniform() < 0.05 and ref.r.__len__() < 200:
                assert lib.add_keyframe() == ref.add_keyframe()
            u = rng.uniform(size=batch).tolist()
            a, b = lib.select(u), ref.select(u)
            assert a == b, (trial, it, a, b)
            for i in a:
                loss = float(rng.choice([rng.uniform(), 0.5]))    # include ties
                lib.report(i, loss)
                ref.report(i, loss)
            assert lib.remaining == ref.r
        assert lib.refills == ref.refills


def test_adaptive_selection_spreads_iterations_over_a_growing_pool():
    """Long-tail effect of Sec. III-C-2: with uniform random re-optimisation
    over a growing pool the oldest keyframes collect far more iterations than
    the newest; the adaptive counts bound every keyframe's share per round."""
    rng = np.random.default_rng(1)
    s = KeyframeScheduler(capacity=512, r0=8, d=4)
    counts_adaptive, counts_random = [], []
    for step in range(4000):
        if step % 20 == 0:
            s.add_keyframe()
            counts_adaptive.append(0)
            counts_random.append(0)
        (i,) = s.select([rng.uniform()])
        counts_adaptive[i] += 1
        s.report(i, float(rng.uniform()))
        counts_random[int(rng.integers(0, len(counts_random)))] += 1
    ca, cr = np.array(counts_adaptive), np.array(counts_random)
    old, new = slice(0, 40), slice(-40, None)
    assert cr[old].mean() / max(cr[new].mean(), 1e-9) > 3.0
    assert ca[old].mean() / max(ca[new].mean(), 1e-9) < cr[old].mean() / max(cr[new].mean(), 1e-9)
