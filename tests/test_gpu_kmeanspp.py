"""GPU K-means++ parity (Sec. 2 D^2 sampling; greedy candidates of Sec. 5;
reseeding of degenerate slots, Sec. 3.3).  Both sides see the same FP32 sample
and centroids, so the D^2 weights are the same FP64 numbers and the picks must
agree exactly: a draw that the GPU's chunked sums leave within rounding of a
running-sum boundary is taken again with W and the running sum added in row
order, as the oracle adds them; a test hook forces that for every draw."""
import numpy as np
import pytest
import torch

import oracle
from paper_2204_07485_amd import synth

pytestmark = pytest.mark.gpu


def _run(P, C, deg, seed, t, trials, grid=0):
    from paper_2204_07485_amd import bigmeans
    Cd = torch.from_numpy(np.ascontiguousarray(C, np.float32)).cuda()
    dg = bigmeans.kmeanspp_seed(torch.from_numpy(P).cuda(), Cd, deg, seed, t,
                                n_local_trials=trials, grid=grid)
    return Cd.cpu().numpy(), dg


@pytest.mark.parametrize("s,d,k,trials,grid", [(50, 2, 5, 1, 0), (2000, 8, 10, 3, 0),
                                               (40_000, 16, 25, 3, 0), (40_000, 16, 25, 1, 7),
                                               (12_345, 68, 50, 3, 0), (3_001, 3, 17, 8, 5),
                                               (10_000, 128, 30, 2, 64)])
def test_full_seeding_matches_oracle(s, d, k, trials, grid):
    print(f"kmeans++ s={s} d={d} k={k} trials={trials} grid={grid}", flush=True)
    P = synth.gaussian_mixture(s, d, k, seed=s + k, sigma_range=(0.5, 2.0))[0]
    C = np.full((k, d), np.nan, np.float32)
    deg = np.ones(k, np.uint8)
    got_C, got_deg = _run(P, C, deg, seed=123, t=4, trials=trials, grid=grid)
    ref_C, ref_deg, _ = oracle.kmeanspp(P, C, deg, seed=123, t=4, trials=trials)
    assert np.array_equal(got_deg, ref_deg)
    assert np.array_equal(got_C, ref_C.astype(np.float32))


def test_partial_reseed_matches_oracle():
    s, d, k = 20_000, 16, 12
    P = synth.gaussian_mixture(s, d, k, seed=3, sigma_range=(0.5, 2.0))[0]
    rng = np.random.default_rng(0)
    C = P[rng.choice(s, k, replace=False)].copy()
    deg = np.zeros(k, np.uint8)
    deg[[0, 4, 5, 11]] = 1
    C[deg == 1] = np.nan
    got_C, got_deg = _run(P, C, deg, seed=9, t=17, trials=3)
    ref_C, ref_deg, _ = oracle.kmeanspp(P, C, deg, seed=9, t=17, trials=3)
    assert np.array_equal(got_deg, ref_deg)
    assert np.array_equal(got_C, ref_C.astype(np.float32))


def test_zero_potential_leaves_slots_degenerate():
    P = np.tile(np.array([[1.5, -2.0, 3.0]], np.float32), (300, 1))
    C = np.full((4, 3), np.nan, np.float32)
    C[1] = P[0]
    deg = np.array([1, 0, 1, 1], np.uint8)
    got_C, got_deg = _run(P, C, deg, seed=1, t=0, trials=3)
    assert got_deg.tolist() == [1, 0, 1, 1]
    assert np.isnan(got_C[[0, 2, 3]]).all()
    assert np.array_equal(got_C[1], P[0])


def test_pick_frequencies_follow_d2_law():
    # first pick uniform, second by D^2, on a tiny input: compare GPU picks with
    # the oracle's picks draw for draw over many sample indices
    P = np.array([[0, 0], [1, 0], [0, 2], [3, 1], [-2, -1], [0.5, 0.5]], np.float32)
    for t in range(200):
        C = np.full((2, 2), np.nan, np.float32)
        got_C, _ = _run(P, C, np.ones(2, np.uint8), seed=55, t=t, trials=3)
        ref_C, _, _ = oracle.kmeanspp(P, C, np.ones(2, np.uint8), seed=55, t=t, trials=3)
        assert np.array_equal(got_C, ref_C.astype(np.float32)), t


@pytest.mark.parametrize("s,d,k,trials,grid", [(2000, 8, 10, 3, 0), (40_000, 16, 25, 3, 0),
                                               (12_345, 68, 50, 3, 0), (3_001, 3, 17, 8, 5),
                                               (65, 2, 6, 1, 1)])
def test_row_order_draws_match_oracle(s, d, k, trials, grid):
    # every draw taken with the row-order sums (the path for draws near a
    # boundary): picks still bit-equal to the oracle's
    from paper_2204_07485_amd import bigmeans
    print(f"kmeans++ row-order draws s={s} d={d} k={k} trials={trials} grid={grid}", flush=True)
    P = synth.gaussian_mixture(s, d, k, seed=s + 2 * k, sigma_range=(0.5, 2.0))[0]
    C = np.full((k, d), np.nan, np.float32)
    deg = np.ones(k, np.uint8)
    prev = bigmeans.debug_exact_draws(1)
    try:
        got_C, got_deg = _run(P, C, deg, seed=77, t=2, trials=trials, grid=grid)
    finally:
        bigmeans.debug_exact_draws(prev)
    ref_C, ref_deg, _ = oracle.kmeanspp(P, C, deg, seed=77, t=2, trials=trials)
    assert np.array_equal(got_deg, ref_deg)
    assert np.array_equal(got_C, ref_C.astype(np.float32))


def test_row_order_draws_with_zero_weights():
    # many rows repeat placed centres (zero weight); the row-order draw skips
    # them exactly as the oracle's running sum does
    from paper_2204_07485_amd import bigmeans
    rng = np.random.default_rng(4)
    base = rng.normal(0, 3, size=(7, 5)).astype(np.float32)
    P = base[rng.integers(0, 7, 5_000)]
    P[::97] += rng.normal(0, 0.01, size=P[::97].shape).astype(np.float32)
    C = np.full((9, 5), np.nan, np.float32)
    deg = np.ones(9, np.uint8)
    prev = bigmeans.debug_exact_draws(1)
    try:
        got_C, got_deg = _run(P, C, deg, seed=3, t=1, trials=3)
    finally:
        bigmeans.debug_exact_draws(prev)
    ref_C, ref_deg, _ = oracle.kmeanspp(P, C, deg, seed=3, t=1, trials=3)
    assert np.array_equal(got_deg, ref_deg)
    got_C[got_deg == 1] = 0
    ref_C[ref_deg == 1] = 0
    assert np.array_equal(got_C, ref_C.astype(np.float32))
