"""GPU assignment parity (Eq. 1 / the assignment step of Sec. 2): labels equal
the oracle's except at near ties, the FP64 objective within 1e-6 relative."""
import numpy as np
import pytest
import torch

import oracle
from paper_2204_07485_amd import synth
from tests.parity import assert_labels, assert_sse

pytestmark = pytest.mark.gpu


def _mixture(n, d, k, seed):
    return synth.gaussian_mixture(n, d, k, seed, sigma_range=(0.5, 2.0), weights="dirichlet")[0]


@pytest.mark.parametrize("n,d,k", [(1, 1, 1), (777, 3, 5), (10_001, 8, 10), (65_537, 16, 25),
                                   (20_000, 68, 50), (9_999, 128, 100), (4_097, 200, 7),
                                   (3_000, 33, 1)])
def test_assign_matches_oracle(n, d, k):
    from paper_2204_07485_amd import bigmeans
    print(f"assign n={n} d={d} k={k}", flush=True)
    X = _mixture(n, d, max(k, 2), seed=n + d)
    rng = np.random.default_rng(k)
    C = X[rng.choice(n, size=k, replace=n < k)].astype(np.float32) + 0.1
    Xd = torch.from_numpy(X).cuda()
    Cd = torch.from_numpy(C).cuda()
    lab, mind, sse = bigmeans.kmeans_assign(Xd, Cd, want_min_d2=True)
    ref_lab, ref_min, ref_sse = oracle.assign(X, C)
    assert_labels(lab.cpu().numpy(), ref_lab, X, C)
    assert_sse(sse, ref_sse)
    same = lab.cpu().numpy() == ref_lab
    np.testing.assert_allclose(mind.cpu().numpy()[same], ref_min[same], rtol=2e-5, atol=1e-6)


def test_assign_skips_degenerate():
    from paper_2204_07485_amd import bigmeans
    X = _mixture(5000, 8, 6, seed=1)
    C = X[:6].copy()
    deg = np.array([0, 1, 0, 1, 0, 0], np.uint8)
    C[deg == 1] = np.nan
    lab, _, sse = bigmeans.kmeans_assign(torch.from_numpy(X).cuda(), torch.from_numpy(C).cuda(), deg)
    lab = lab.cpu().numpy()
    assert not np.isin(lab, [1, 3]).any()
    ref_lab, _, ref_sse = oracle.assign(X, C, deg)
    assert_labels(lab, ref_lab, X, C, deg)
    assert_sse(sse, ref_sse)


def test_assign_exact_ties_go_to_lowest_index():
    from paper_2204_07485_amd import bigmeans
    X = np.array([[0.0, 0.0], [1.0, 1.0], [2.0, 0.0]], np.float32)
    C = np.array([[1.0, 0.0], [1.0, 0.0], [-1.0, 0.0], [3.0, 0.0]], np.float32)
    lab, _, _ = bigmeans.kmeans_assign(torch.from_numpy(X).cuda(), torch.from_numpy(C).cuda())
    assert lab.cpu().tolist() == [0, 0, 0]


def test_assign_bf16_input():
    from paper_2204_07485_amd import bigmeans
    X = _mixture(40_000, 128, 20, seed=4)
    H = synth.to_bf16_bits(X)
    Xf = synth.bf16_bits_to_f32(H)
    C = Xf[:20].copy()
    Hd = torch.from_numpy(H.view(np.int16)).cuda()
    lab, _, sse = bigmeans.kmeans_assign(Hd, torch.from_numpy(C).cuda())
    ref_lab, _, ref_sse = oracle.assign(Xf, C)
    assert_labels(lab.cpu().numpy(), ref_lab, Xf, C)
    assert_sse(sse, ref_sse)


def test_assign_full_medium_workload():
    # the final pass of the medium workload at full size (1,000,000 x 16, k=25),
    # in the launch configuration the benchmark times
    from paper_2204_07485_amd import bigmeans
    X = synth.make_medium()
    C = X[np.random.default_rng(0).choice(len(X), 25, replace=False)] + 0.25
    lab, _, sse = bigmeans.kmeans_assign(torch.from_numpy(X).cuda(), torch.from_numpy(C).cuda())
    ref_lab, _, ref_sse = oracle.assign(X, C)
    assert_sse(sse, ref_sse)
    assert_labels(lab.cpu().numpy(), ref_lab, X, C)


def test_assign_fp32_centroids_beyond_64k_lds():
    # k x d = 128 x 128 FP32 centroids (64 KiB + flags) need the large-LDS launch attribute
    from paper_2204_07485_amd import bigmeans
    X = _mixture(30_000, 128, 128, seed=9)
    C = X[np.random.default_rng(9).choice(len(X), 128, replace=False)].astype(np.float32) + 0.1
    lab, _, sse = bigmeans.kmeans_assign(torch.from_numpy(X).cuda(), torch.from_numpy(C).cuda())
    ref_lab, _, ref_sse = oracle.assign(X, C)
    assert_labels(lab.cpu().numpy(), ref_lab, X, C)
    assert_sse(sse, ref_sse)


def test_assign_nonfinite_rows_get_a_valid_label():
    # a row with a NaN or an infinite coordinate has no nearest centroid; it
    # still gets an active slot, and the other rows are unaffected
    from paper_2204_07485_amd import bigmeans
    X = _mixture(2_000, 8, 4, seed=10)
    X[5, 3] = np.nan
    X[17, 0] = np.inf
    C = X[[0, 1, 2, 3]].copy()
    deg = np.array([1, 0, 0, 0], np.uint8)
    lab, _, _ = bigmeans.kmeans_assign(torch.from_numpy(X).cuda(), torch.from_numpy(C).cuda(), deg)
    lab = lab.cpu().numpy()
    assert lab[5] == 1 and lab[17] == 1
    ok = np.ones(len(X), bool)
    ok[[5, 17]] = False
    ref_lab, _, _ = oracle.assign(X[ok], C, deg)
    assert_labels(lab[ok], ref_lab, X[ok], C, deg)
