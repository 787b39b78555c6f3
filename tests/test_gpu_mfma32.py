"""GPU parity of the FP32 matrix-core assignment (the full-data pass for FP32
X with d >= 8, k >= 8 and k d >= 256; every case below meets that).

Its labels must equal the VALU FP32 direct-difference kernel's bit for bit
(the error band and the FP32 recheck make them so; the test hook
debug_fp32_mfma(0) runs the VALU kernel); against the FP64 oracle they follow
the same near-tie rule as the FP32 path.  Its objective terms are the FP64
squared distances of the chosen centroids, summed in another association, so
the objective agrees with the VALU kernel's to 1e-12 and with the oracle to
1e-6.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2204_07485_amd import synth
from tests.parity import assert_labels, assert_sse

pytestmark = pytest.mark.gpu


def _mixture(n, d, k, seed, offset=0.0):
    X, _ = synth.gaussian_mixture(n, d, max(k, 2), seed, sigma_range=(0.5, 2.0), outlier_frac=0.1)
    return (X + offset).astype(np.float32)


def _centroids(X, k, seed, jitter=0.05):
    rng = np.random.default_rng(seed)
    C = X[rng.choice(len(X), size=k, replace=len(X) < k)].astype(np.float64)
    return (C + rng.normal(0.0, jitter, C.shape)).astype(np.float32)


def _both(Xd, Cd, deg=None):
    """(matrix-core result, VALU result) of kmeans_assign."""
    from paper_2204_07485_amd import bigmeans
    prev = bigmeans.debug_fp32_mfma(0)
    try:
        ref = bigmeans.kmeans_assign(Xd, Cd, deg, want_min_d2=True)
    finally:
        bigmeans.debug_fp32_mfma(prev)
    assert prev == 1
    got = bigmeans.kmeans_assign(Xd, Cd, deg, want_min_d2=True)
    return got, ref


def _check_equal(got, ref, sse_rel=1e-12):
    lab, mind, sse = got
    rlab, rmind, rsse = ref
    np.testing.assert_array_equal(lab.cpu().numpy(), rlab.cpu().numpy())
    if np.isfinite(rsse):
        assert abs(sse - rsse) <= sse_rel * abs(rsse) + 1e-300, (sse, rsse)
    np.testing.assert_allclose(mind.cpu().numpy(), rmind.cpu().numpy(), rtol=1e-6, atol=0)


@pytest.mark.parametrize("n,d,k", [(1, 8, 128), (33, 8, 128), (10_001, 16, 64), (20_000, 68, 50),
                                   (60_013, 128, 100), (4_097, 200, 17), (3_001, 256, 64),
                                   (5_000, 40, 128), (2_048, 36, 29), (2_000, 203, 9),
                                   (7_777, 80, 33)])
def test_mfma32_matches_valu_path_and_oracle(n, d, k):
    X = _mixture(n, d, k, seed=n + d)
    C = _centroids(X, k, seed=k)
    print(f"mfma32 n={n} d={d} k={k}", flush=True)
    got, ref = _both(torch.from_numpy(X).cuda(), torch.from_numpy(C).cuda())
    _check_equal(got, ref)
    olab, _, osse = oracle.assign(X, C)
    assert_labels(got[0].cpu().numpy(), olab, X, C)
    assert_sse(got[2], osse)


def test_mfma32_near_ties_follow_fp32_rounding():
    # points moved onto the bisector hyperplanes of centroid pairs: their two
    # distances agree to within rounding, so the FP32 path's own rounding
    # decides the label and the recheck must reproduce it
    rng = np.random.default_rng(21)
    d, k, n = 32, 32, 8_192
    C = rng.uniform(-10, 10, size=(k, d)).astype(np.float32)
    a = rng.integers(0, k, n)
    b = (a + 1 + rng.integers(0, k - 1, n)) % k
    x = rng.uniform(-10, 10, size=(n, d))
    u = C[a].astype(np.float64) - C[b]
    mid = 0.5 * (C[a].astype(np.float64) + C[b])
    x -= (((x - mid) * u).sum(1) / (u * u).sum(1))[:, None] * u
    X = x.astype(np.float32)
    got, ref = _both(torch.from_numpy(X).cuda(), torch.from_numpy(C).cuda())
    _check_equal(got, ref)


def test_mfma32_exact_ties_and_degenerate_slots():
    # duplicated centroid rows tie exactly: the lowest index wins; degenerate
    # slots (NaN rows, flagged) are never chosen
    X = _mixture(6_000, 24, 48, seed=3)
    C = _centroids(X, 48, seed=4)
    C[7] = C[2]
    C[11] = C[5]
    deg = np.zeros(48, np.uint8)
    deg[[0, 9]] = 1
    C[[0, 9]] = np.nan
    got, ref = _both(torch.from_numpy(X).cuda(), torch.from_numpy(C).cuda(), deg)
    _check_equal(got, ref)
    lab = got[0].cpu().numpy()
    assert not np.isin(lab, [0, 9, 7, 11]).any()


def test_mfma32_far_from_the_origin():
    # |x| much larger than the distances: the band is wide relative to the
    # gaps and many points take the recheck
    X = _mixture(20_000, 16, 64, seed=8, offset=3.0e3)
    C = _centroids(X, 64, seed=9)
    got, ref = _both(torch.from_numpy(X).cuda(), torch.from_numpy(C).cuda())
    _check_equal(got, ref)


def test_mfma32_nonfinite_rows_and_unaligned_view():
    # rows with NaN or infinite coordinates get the VALU kernel's label (the
    # first active slot); an X view 4 bytes into its buffer takes the
    # element-wise load path
    X = _mixture(3_000, 20, 52, seed=12)
    X[5, 3] = np.nan
    X[17, 0] = np.inf
    X[99, 19] = -np.inf
    C = _centroids(X[100:], 52, seed=13)
    flat = torch.from_numpy(np.concatenate([[0.0], X.reshape(-1)]).astype(np.float32)).cuda()
    Xd = flat[1:].view(3_000, 20)
    assert Xd.data_ptr() % 16 != 0
    deg = np.zeros(52, np.uint8)
    deg[0] = 1
    got, ref = _both(Xd, torch.from_numpy(C).cuda(), deg)
    lab, rlab = got[0].cpu().numpy(), ref[0].cpu().numpy()
    np.testing.assert_array_equal(lab, rlab)
    assert lab[5] == 1 and lab[17] == 1 and lab[99] == 1
    ok = np.ones(len(X), bool)
    ok[[5, 17, 99]] = False
    mind, rmind = got[1].cpu().numpy(), ref[1].cpu().numpy()
    np.testing.assert_allclose(mind[ok], rmind[ok], rtol=1e-6, atol=0)
    assert np.isnan(mind[5]) and np.isnan(rmind[5])
    assert np.isinf(mind[17]) and np.isinf(rmind[17])


def test_mfma32_in_a_fit_final_pass():
    # a fit's full-data pass (400,000 x 68, k = 50) on the matrix cores: the
    # fit's labels and objective equal the VALU kernel's on the fitted centroids
    from paper_2204_07485_amd import bigmeans
    X = torch.from_numpy(_mixture(400_000, 68, 50, seed=17)).cuda()
    r = bigmeans.bigmeans_fit(X, 50, 20_000, 3, 7, max_iter=300, tol=1e-4,
                              stop_rule=bigmeans.BM_STOP_REL_OBJ)
    got, ref = _both(X, r["centroids"], r["degenerate"])
    _check_equal(got, ref)
    np.testing.assert_array_equal(r["labels"].cpu().numpy(), ref[0].cpu().numpy())
    assert abs(r["sse"] - ref[2]) <= 1e-12 * ref[2]
