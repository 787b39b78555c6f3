"""Pins for the oracle's functions beyond the sequential Big-means loop:

- the Forgy-style (re)initialisation (Sec. 3.3 allows initialisations other
  than K-means++): every degenerate slot takes a uniformly drawn row, slots
  independently (chi-square on the exact laws), active slots untouched, and its
  first draw is the draw K-means++ uses for its uniform first centre;
- collective parallel Big-means (Sec. 3.6, third scheme): one worker is Alg. 1
  itself; every worker's result is a one-sample Alg. 1 step from the round's
  incumbent; the incumbent is the running minimum over rounds of the per-round
  best worker; never below the brute-force optimum on tiny inputs;
- the sample-size rule of thumb (Sec. 5): the sizes it tries, the objectives it
  sees (each a full Big-means run) and where it stops.
"""
import numpy as np
import pytest
from scipy import stats

import oracle
from tests.brute import brute_force_opt


def _separated(n_per, centers, sigma, seed):
    rng = np.random.default_rng(seed)
    pts = [np.asarray(c, float) + sigma * rng.normal(size=(n_per, len(c))) for c in centers]
    return np.concatenate(pts).astype(np.float32)


def _mixture(n, d, comps, seed, sigma=1.0, spread=6.0):
    rng = np.random.default_rng(seed)
    mu = rng.uniform(-spread, spread, size=(comps, d))
    lab = rng.integers(0, comps, size=n)
    return (mu[lab] + sigma * rng.normal(size=(n, d))).astype(np.float32)


# -------------------------------------------------------------------- Forgy

def test_forgy_pick_is_uniform():
    P = np.arange(6, dtype=np.float64).reshape(6, 1) * 10.0
    C = np.array([[5.0], [np.nan], [15.0]])
    deg = np.array([0, 1, 0], np.uint8)
    picks = []
    for seed in range(1, 3001):
        Cn, dn, st = oracle.forgy(P, C, deg, seed=seed, t=7)
        assert dn.tolist() == [0, 0, 0]
        assert Cn[0, 0] == 5.0 and Cn[2, 0] == 15.0       # active slots untouched
        assert st["reseeded"] == 1 and st["n_d"] == 0
        picks.append(int(Cn[1, 0] // 10))
    counts = np.bincount(picks, minlength=6)
    assert stats.chisquare(counts).pvalue > 1e-3


def test_forgy_slots_are_independent_draws():
    P = np.arange(6, dtype=np.float64).reshape(6, 1)
    C = np.full((2, 1), np.nan)
    cells = []
    for seed in range(1, 7201):
        Cn, _, _ = oracle.forgy(P, C, [1, 1], seed=seed, t=0)
        cells.append(int(Cn[0, 0]) * 6 + int(Cn[1, 0]))
    counts = np.bincount(cells, minlength=36)
    assert stats.chisquare(counts).pvalue > 1e-3
    assert counts[::7].sum() > 0        # the same row twice is possible


def test_forgy_first_draw_is_kmeanspp_uniform_first_centre():
    rng = np.random.default_rng(3)
    P = rng.normal(size=(50, 3))
    for seed in range(1, 40):
        a, _, _ = oracle.forgy(P, np.zeros((4, 3)), np.ones(4, np.uint8), seed=seed, t=2)
        b, _, _ = oracle.kmeanspp(P, np.zeros((4, 3)), np.ones(4, np.uint8), seed=seed, t=2)
        assert np.array_equal(a[0], b[0])


def test_bigmeans_forgy_keeps_the_best_and_respects_the_optimum():
    X = _separated(4, [[0, 0], [5, 5], [0, 6]], 0.5, seed=4)  # n = 12
    opt = brute_force_opt(X.astype(np.float64), 3)
    r = oracle.bigmeans_fit(X, 3, 8, 12, seed=6, init_method=oracle.ORC_INIT_FORGY)
    assert r["sse"] >= opt - 1e-9
    assert r["f_opt"] == r["sample_f"].min()
    r2 = oracle.bigmeans_fit(X, 3, 8, 12, seed=6)
    assert not np.array_equal(r["sample_f"], r2["sample_f"])   # a different initialiser


# --------------------------------------------------------------- collective

def test_collective_with_one_worker_is_alg1():
    X = _mixture(3000, 4, 6, seed=11)
    a = oracle.bigmeans_collective(X, 6, 400, 1, 9, seed=21)
    b = oracle.bigmeans_fit(X, 6, 400, 9, seed=21)
    assert np.array_equal(a["worker_f"][:, 0], b["sample_f"])
    assert np.array_equal(a["C"], b["C"], equal_nan=True)
    assert a["sse"] == b["sse"] and a["f_opt"] == b["f_opt"]
    assert np.array_equal(a["labels"], b["labels"])
    assert a["stats"] == b["stats"]


def test_collective_workers_start_from_the_round_incumbent():
    X = _mixture(4000, 3, 7, seed=12, sigma=1.3)
    W, R, k, s, seed = 3, 4, 7, 300, 5
    full = oracle.bigmeans_collective(X, k, s, W, R, seed)
    state = None
    running = np.inf
    repl = 0
    for r in range(R):
        if r > 0:
            prev = oracle.bigmeans_collective(X, k, s, W, r, seed, want_labels=False)
            state = (prev["C"], prev["deg"], prev["f_opt"])
            assert prev["f_opt"] == running
        for w in range(W):
            one = oracle.bigmeans_fit(X, k, s, 1, seed, t_start=r * W + w, state=state,
                                      want_labels=False, want_sse=False)
            assert one["sample_f"][0] == full["worker_f"][r, w], (r, w)
        best = full["worker_f"][r].min()
        if best < running:
            running = best
            repl += 1
    assert full["f_opt"] == running == full["worker_f"].min()
    assert full["stats"]["replacements"] == repl
    assert full["stats"]["samples"] == W * R


def test_collective_never_below_brute_force_optimum():
    X = _separated(4, [[0, 0], [4, 1], [1, 5]], 0.7, seed=13)
    opt = brute_force_opt(X.astype(np.float64), 3)
    r = oracle.bigmeans_collective(X, 3, 9, 4, 3, seed=2)
    assert r["sse"] >= opt - 1e-9
    r = oracle.bigmeans_collective(X, 3, 12, 4, 2, seed=2)
    assert r["sse"] == pytest.approx(opt, rel=1e-12)


# ------------------------------------------------------------ sample sizes

def test_sample_size_sweep_replays():
    X = _mixture(8000, 2, 25, seed=16, sigma=0.5, spread=20)
    best, tried = oracle.sample_size_sweep(X, 25, 30, 8000, 3, seed=3)
    sizes = [s for s, _ in tried]
    sse = [v for _, v in tried]
    assert sizes == [30 * 2 ** i for i in range(len(sizes))] and len(sizes) >= 4
    for s, v in tried:   # each objective is a full Big-means run at that size
        assert v == oracle.bigmeans_fit(X, 25, s, 3, seed=3, want_labels=False)["sse"]
    # strictly decreasing until the last size tried, which is the first one
    # that does not improve (it stopped before the cap)
    for i in range(1, len(sse) - 1):
        assert sse[i] < sse[i - 1]
    assert sse[-1] >= min(sse[:-1])
    assert best == sizes[int(np.argmin(sse))] == sizes[-2]


def test_sample_size_sweep_reaches_the_cap():
    X = _mixture(500, 2, 4, seed=15)
    best, tried = oracle.sample_size_sweep(X, 4, 400, 500, 2, seed=3)
    assert [s for s, _ in tried][:2] == [400, 500]
    assert best in (400, 500)


def test_collective_round_ties_go_to_the_lowest_worker():
    # k = s = n distinct points: every worker reaches f = 0 with its own slot
    # order, so the round is a tie of all workers and the lowest one wins
    X = np.array([[0, 0], [3, 1], [7, 2], [1, 9], [5, 5]], np.float32)
    r = oracle.bigmeans_collective(X, 5, 5, 3, 1, seed=8)
    assert (r["worker_f"] == 0).all()
    w0 = oracle.bigmeans_fit(X, 5, 5, 1, seed=8, want_labels=False)
    w1 = oracle.bigmeans_fit(X, 5, 5, 1, seed=8, t_start=1, want_labels=False)
    assert not np.array_equal(w0["C"], w1["C"])
    assert np.array_equal(r["C"], w0["C"])


def test_sample_size_sweep_stops_on_an_equal_objective():
    # three distinct values, ten copies each: every size finds them exactly
    # (objective 0), so the second size does not improve and the sweep stops
    X = np.repeat(np.array([[0, 0], [4, 0], [0, 4]], np.float32), 10, axis=0)
    best, tried = oracle.sample_size_sweep(X, 3, 6, 30, 3, seed=2)
    assert tried == [(6, 0.0), (12, 0.0)]
    assert best == 6
