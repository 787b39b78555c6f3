"""Pins for the oracle's K-means++ (Sec. 2: D^2 sampling; Sec. 5: greedy form
with three candidates; Sec. 3.3: only degenerate slots are (re)initialised).

The exact laws are enumerated here with independent numpy arithmetic and
compared with empirical pick frequencies over many sample indices t."""
import itertools
import math

import numpy as np
import pytest
from scipy import stats

import oracle
from tests.brute import brute_force_opt


def _d2(a, b):
    return float(((np.asarray(a, float) - np.asarray(b, float)) ** 2).sum())


P6 = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 2.0], [3.0, 1.0], [-2.0, -1.0], [0.5, 0.5]])
C_ACTIVE = np.array([0.2, 0.1])


def _pick(P, C, deg, t, trials, slot):
    Cn, degn, _ = oracle.kmeanspp(P, C, deg, seed=314, t=t, trials=trials)
    assert degn[slot] == 0
    row = Cn[slot]
    hits = np.where((P == row).all(axis=1))[0]
    assert len(hits) >= 1
    return int(hits[0])


def _chi2_ok(counts, probs, reps):
    keep = probs > 0
    assert counts[~keep].sum() == 0
    exp = probs[keep] * reps
    return stats.chisquare(counts[keep], exp * counts[keep].sum() / exp.sum()).pvalue > 1e-4


def test_first_centre_is_uniform():
    reps = 12000
    C = np.full((1, 2), np.nan)
    counts = np.zeros(6)
    for t in range(reps):
        counts[_pick(P6, C, [1], t, 3, 0)] += 1
    assert _chi2_ok(counts, np.full(6, 1 / 6), reps)


def test_d2_law_single_candidate():
    reps = 20000
    C = np.array([C_ACTIVE, [np.nan, np.nan]])
    w = np.array([_d2(p, C_ACTIVE) for p in P6])
    counts = np.zeros(6)
    for t in range(reps):
        counts[_pick(P6, C, [0, 1], t, 1, 1)] += 1
    assert _chi2_ok(counts, w / w.sum(), reps)


def _greedy_law(P, centre, trials):
    w = np.array([_d2(p, centre) for p in P])
    pw = w / w.sum()
    phi = np.array([sum(min(w[i], _d2(P[i], P[c])) for i in range(len(P))) for c in range(len(P))])
    law = np.zeros(len(P))
    for tri in itertools.product(range(len(P)), repeat=trials):
        prob = np.prod([pw[c] for c in tri])
        if prob == 0:
            continue
        best = tri[0]
        for c in tri[1:]:
            if phi[c] < phi[best]:
                best = c
        law[best] += prob
    return law


def test_greedy_three_candidate_law():
    reps = 20000
    C = np.array([C_ACTIVE, [np.nan, np.nan]])
    law = _greedy_law(P6, C_ACTIVE, 3)
    counts = np.zeros(6)
    for t in range(reps):
        counts[_pick(P6, C, [0, 1], t, 3, 1)] += 1
    assert _chi2_ok(counts, law, reps)
    # the greedy law differs from plain D^2 sampling on this input
    w = np.array([_d2(p, C_ACTIVE) for p in P6])
    assert np.abs(law - w / w.sum()).max() > 0.05


def test_slots_filled_in_ascending_order_with_updated_weights():
    # deg = [1, 0, 1]: slot 0 is drawn by D^2 to the active slot 1, then slot 2
    # by D^2 to {slot 1, slot 0}.  Joint law enumerated exactly.
    reps = 20000
    C = np.array([[np.nan, np.nan], C_ACTIVE, [np.nan, np.nan]])
    w1 = np.array([_d2(p, C_ACTIVE) for p in P6])
    joint = np.zeros((6, 6))
    for a in range(6):
        if w1[a] == 0:
            continue
        w2 = np.minimum(w1, [_d2(p, P6[a]) for p in P6])
        if w2.sum() == 0:
            continue
        joint[a] = (w1[a] / w1.sum()) * (w2 / w2.sum())
    counts = np.zeros((6, 6))
    for t in range(reps):
        Cn, degn, _ = oracle.kmeanspp(P6, C, [1, 0, 1], seed=5, t=t, trials=1)
        assert list(degn) == [0, 0, 0]
        assert np.array_equal(Cn[1], C_ACTIVE)
        a = int(np.where((P6 == Cn[0]).all(axis=1))[0][0])
        b = int(np.where((P6 == Cn[2]).all(axis=1))[0][0])
        counts[a, b] += 1
    assert _chi2_ok(counts.ravel(), joint.ravel(), reps)


def test_zero_potential_leaves_slots_degenerate():
    P = np.tile([[1.0, 2.0]], (5, 1))
    C = np.array([[1.0, 2.0], [np.nan, np.nan], [np.nan, np.nan]])
    Cn, degn, st = oracle.kmeanspp(P, C, [0, 1, 1], seed=1, t=0)
    assert list(degn) == [0, 1, 1]
    assert np.isnan(Cn[1:]).all()
    assert st["reseeded"] == 0


def test_active_slots_untouched():
    rng = np.random.default_rng(0)
    P = rng.normal(size=(50, 3))
    C = rng.normal(size=(4, 3))
    C[2] = np.nan
    Cn, degn, st = oracle.kmeanspp(P, C, [0, 0, 1, 0], seed=3, t=1)
    assert np.array_equal(Cn[[0, 1, 3]], C[[0, 1, 3]])
    assert st["reseeded"] == 1
    assert any((P == Cn[2]).all(axis=1))


def test_seeding_cost_bound():
    # Sec. 2 quotes E[cost] <= 5 (log k + 2) OPT for K-means++; checked on a
    # brute-forced tiny input (natural log).  A weak, expectation-level pin.
    rng = np.random.default_rng(8)
    P = np.concatenate([rng.normal(c, 0.3, size=(3, 2)) for c in ([0, 0], [4, 0], [0, 5])])
    k = 3
    opt = brute_force_opt(P, k)
    costs = []
    for t in range(3000):
        Cn, degn, _ = oracle.kmeanspp(P, np.full((k, 2), np.nan), [1] * k, seed=17, t=t, trials=1)
        costs.append(oracle.assign(P, Cn, degn)[2])
    assert np.mean(costs) <= 5 * (math.log(k) + 2) * opt
