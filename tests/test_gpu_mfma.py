"""GPU parity of the BF16 matrix-core assignment (BM_PREC_BF16_MFMA).

Its labels must equal the FP32 direct-difference path's bit for bit (the
near-tie recheck makes them so); against the FP64 oracle they follow the
same near-tie rule as the FP32 path.  Its objective terms are FP32 sums of 8
squared differences added in FP64 (within 6e-7 relative of the exact terms),
so the objective of Eq. (1) is checked to 1e-6 against the oracle and the FP32
path, and the per-point distances to 1e-6 against the FP32 path's.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2204_07485_amd import synth
from tests.parity import assert_labels, assert_sse

pytestmark = pytest.mark.gpu


def _bf16_mixture(n, d, k, seed, outliers=0.1):
    X, _ = synth.gaussian_mixture(n, d, max(k, 2), seed, sigma_range=(0.5, 2.0),
                                  outlier_frac=outliers)
    H = synth.to_bf16_bits(X)
    return H, synth.bf16_bits_to_f32(H)


def _centroids(Xf, k, seed, jitter=0.05):
    rng = np.random.default_rng(seed)
    C = Xf[rng.choice(len(Xf), size=k, replace=len(Xf) < k)].astype(np.float64)
    return (C + rng.normal(0.0, jitter, C.shape)).astype(np.float32)


def _both(H, C, deg=None, min_d2=True):
    from paper_2204_07485_amd import bigmeans
    Hd = torch.from_numpy(H.view(np.int16)).cuda()
    Cd = torch.from_numpy(C).cuda()
    ref = bigmeans.kmeans_assign(Hd, Cd, deg, want_min_d2=min_d2)
    got = bigmeans.kmeans_assign(Hd, Cd, deg, want_min_d2=min_d2,
                                 precision=bigmeans.BM_PREC_BF16_MFMA)
    return got, ref, bigmeans.last_rechecked()


def _check_equal_to_fp32_path(got, ref):
    lab, mind, sse = got
    rlab, rmind, rsse = ref
    np.testing.assert_array_equal(lab.cpu().numpy(), rlab.cpu().numpy())
    assert abs(sse - rsse) <= 1e-6 * abs(rsse) + 1e-300
    if mind is not None:
        np.testing.assert_allclose(mind.cpu().numpy(), rmind.cpu().numpy(), rtol=1e-6, atol=0)


@pytest.mark.parametrize("n,d,k", [(1, 1, 1), (31, 2, 3), (33, 8, 5), (10_001, 16, 25),
                                   (20_000, 68, 50), (60_013, 128, 100), (4_097, 200, 7),
                                   (3_001, 256, 64), (5_000, 40, 128), (2_048, 33, 17),
                                   (2_000, 203, 9)])
def test_mfma_assign_matches_fp32_path_and_oracle(n, d, k):
    print(f"mfma assign n={n} d={d} k={k}", flush=True)
    H, Xf = _bf16_mixture(n, d, k, seed=n + d + k)
    C = _centroids(Xf, k, seed=k)
    got, ref, nre = _both(H, C)
    _check_equal_to_fp32_path(got, ref)
    ref_lab, _, ref_sse = oracle.assign(Xf, C)
    assert_labels(got[0].cpu().numpy(), ref_lab, Xf, C)
    assert_sse(got[2], ref_sse)
    assert 0 <= nre <= n


def test_mfma_degenerate_centroids_are_skipped():
    H, Xf = _bf16_mixture(12_345, 128, 40, seed=9)
    C = _centroids(Xf, 40, seed=2)
    deg = np.zeros(40, np.uint8)
    deg[[0, 5, 17, 39]] = 1
    C[deg == 1] = np.nan
    got, ref, _ = _both(H, C, deg)
    _check_equal_to_fp32_path(got, ref)
    assert not np.isin(got[0].cpu().numpy(), [0, 5, 17, 39]).any()
    ref_lab, _, ref_sse = oracle.assign(Xf, C, deg)
    assert_labels(got[0].cpu().numpy(), ref_lab, Xf, C, deg)
    assert_sse(got[2], ref_sse)


def test_mfma_exact_ties_go_to_lowest_index():
    # duplicated centroids: every point is an exact tie between the copies,
    # so every point goes through the recheck and takes the lower index
    H, Xf = _bf16_mixture(4_000, 64, 8, seed=3, outliers=0.0)
    C0 = _centroids(Xf, 8, seed=1)
    C = np.concatenate([C0, C0])[np.r_[8:16, 0:8]].copy()  # copies at j and j + 8
    got, ref, nre = _both(H, C)
    _check_equal_to_fp32_path(got, ref)
    assert (got[0].cpu().numpy() < 8).all()
    assert nre == 4_000


def test_mfma_near_ties_follow_fp32_rounding():
    # points rounded onto the bisector hyperplanes of centroid pairs: their
    # two distances agree to within rounding, so the FP32 path's own rounding
    # decides the label and the recheck must reproduce it
    rng = np.random.default_rng(11)
    d, k = 128, 32
    C = rng.uniform(-10, 10, size=(k, d)).astype(np.float32)
    n = 8_192
    a = rng.integers(0, k, n)
    b = (a + 1 + rng.integers(0, k - 1, n)) % k
    x = rng.uniform(-10, 10, size=(n, d))
    u = C[a].astype(np.float64) - C[b]
    mid = 0.5 * (C[a].astype(np.float64) + C[b])
    x -= (((x - mid) * u).sum(1) / (u * u).sum(1))[:, None] * u
    H = synth.to_bf16_bits(x.astype(np.float32))
    got, ref, nre = _both(H, C)
    _check_equal_to_fp32_path(got, ref)
    assert nre > 0


def test_mfma_unaligned_and_odd_rows():
    # d not a multiple of 8 and an X view that starts 2 bytes into its buffer:
    # the kernel takes its element-wise load path
    from paper_2204_07485_amd import bigmeans
    H, Xf = _bf16_mixture(3_001, 24, 6, seed=5)
    C = _centroids(Xf, 6, seed=6)
    flat = torch.from_numpy(np.concatenate([[0], H.reshape(-1)]).astype(np.uint16).view(np.int16)).cuda()
    Hd = flat[1:].view(3_001, 24)
    assert Hd.data_ptr() % 16 != 0
    Cd = torch.from_numpy(C).cuda()
    lab, _, sse = bigmeans.kmeans_assign(Hd, Cd, precision=bigmeans.BM_PREC_BF16_MFMA)
    rlab, _, rsse = bigmeans.kmeans_assign(Hd, Cd)
    np.testing.assert_array_equal(lab.cpu().numpy(), rlab.cpu().numpy())
    assert abs(sse - rsse) <= 1e-6 * rsse


def test_mfma_rejects_bad_requests():
    from paper_2204_07485_amd import bigmeans
    X = torch.zeros((64, 8), dtype=torch.float32, device="cuda")
    C = torch.zeros((4, 8), dtype=torch.float32, device="cuda")
    with pytest.raises(bigmeans.BigmeansError) as e:
        bigmeans.kmeans_assign(X, C, precision=bigmeans.BM_PREC_BF16_MFMA)
    assert e.value.code == bigmeans.BM_EINVAL
    Hb = torch.zeros((64, 300), dtype=torch.int16, device="cuda")
    with pytest.raises(bigmeans.BigmeansError) as e:
        bigmeans.kmeans_assign(Hb, torch.zeros((4, 300), dtype=torch.float32, device="cuda"),
                               precision=bigmeans.BM_PREC_BF16_MFMA)
    assert e.value.code == bigmeans.BM_ENOTSUP
    Hk = torch.zeros((64, 8), dtype=torch.int16, device="cuda")
    with pytest.raises(bigmeans.BigmeansError) as e:
        bigmeans.kmeans_assign(Hk, torch.zeros((129, 8), dtype=torch.float32, device="cuda"),
                               precision=bigmeans.BM_PREC_BF16_MFMA)
    assert e.value.code == bigmeans.BM_ENOTSUP


def test_mfma_full_bf16_workload():
    # the final pass of the BF16 workload at full size (5,000,000 x 128, k=100):
    # bit-equal labels with the FP32 path, and sampled rows against the oracle
    from paper_2204_07485_amd import bigmeans
    H = synth.make_bf16()
    Xf_s = None
    rng = np.random.default_rng(0)
    rows = rng.choice(len(H), 100, replace=False)
    C = (synth.bf16_bits_to_f32(H[rows]).astype(np.float64)
         + rng.normal(0, 0.05, (100, 128))).astype(np.float32)
    Hd = torch.from_numpy(H.view(np.int16)).cuda()
    Cd = torch.from_numpy(C).cuda()
    lab, _, sse = bigmeans.kmeans_assign(Hd, Cd, precision=bigmeans.BM_PREC_BF16_MFMA)
    nre = bigmeans.last_rechecked()
    rlab, _, rsse = bigmeans.kmeans_assign(Hd, Cd)
    lab = lab.cpu().numpy()
    np.testing.assert_array_equal(lab, rlab.cpu().numpy())
    assert abs(sse - rsse) <= 1e-6 * rsse
    assert nre < len(H) // 50, f"{nre} rechecks"
    sample = rng.choice(len(H), 20_000, replace=False)
    Xf_s = synth.bf16_bits_to_f32(H[sample])
    ref_lab, _, _ = oracle.assign(Xf_s, C)
    assert_labels(lab[sample], ref_lab, Xf_s, C)


def test_fit_final_pass_mfma():
    # bigmeans_fit with the MFMA final pass: labels equal the FP32 path's
    # assignment to the returned centroids, SSE likewise
    from paper_2204_07485_amd import bigmeans
    H, Xf = _bf16_mixture(50_000, 128, 20, seed=21)
    Hd = torch.from_numpy(H.view(np.int16)).cuda()
    r = bigmeans.bigmeans_fit(Hd, 20, 5_000, 4, 77, precision=bigmeans.BM_PREC_BF16_MFMA)
    lab, _, sse = bigmeans.kmeans_assign(Hd, r["centroids"], r["degenerate"])
    np.testing.assert_array_equal(r["labels"].cpu().numpy(), lab.cpu().numpy())
    assert abs(r["sse"] - sse) <= 1e-6 * sse
    assert r["stats"]["rechecked"] >= 0


@pytest.mark.parametrize("d,k,init", [(32, 10, 0), (40, 12, 0), (128, 30, 1)])
def test_fit_sample_lloyd_on_matrix_cores_matches_oracle(d, k, init):
    # BM_PREC_BF16_MFMA fits run the sample-level K-means on the matrix cores
    # (labels equal to the FP32 path's); the whole fit must meet the oracle's
    # bar, and agree with the same fit on the FP32 persistent solver
    from paper_2204_07485_amd import bigmeans
    from tests.parity import assert_centroids, assert_labels, assert_sse
    X, _ = synth.gaussian_mixture(60_000, d, k, seed=13 + d, sigma_range=(0.5, 2.0),
                                  outlier_frac=0.1)
    H = synth.to_bf16_bits(X)
    Hd = torch.from_numpy(H.view(np.int16)).cuda()
    kw = dict(stop_rule=bigmeans.BM_STOP_REL_OBJ, max_iter=300, init_method=init)
    print(f"mfma sample lloyd d={d} k={k} init={init}", flush=True)
    got = bigmeans.bigmeans_fit(Hd, k, 6000, 5, 2, sample_idx=True,
                                precision=bigmeans.BM_PREC_BF16_MFMA, **kw)
    prev = bigmeans.debug_mfma_lloyd(0)
    try:
        alt = bigmeans.bigmeans_fit(Hd, k, 6000, 5, 2, precision=bigmeans.BM_PREC_BF16_MFMA, **kw)
    finally:
        bigmeans.debug_mfma_lloyd(prev)
    ref = oracle.bigmeans_fit(H, k, 6000, 5, 2, want_sample_idx=True,
                              stop_rule=oracle.ORC_STOP_REL_OBJ, max_iter=300, init_method=init)
    Xf = synth.bf16_bits_to_f32(H)
    assert np.array_equal(got["sample_idx"].cpu().numpy(), ref["sample_idx"])
    np.testing.assert_allclose(got["sample_f"], ref["sample_f"], rtol=1e-6)
    np.testing.assert_allclose(got["sample_f"], alt["sample_f"], rtol=1e-6)
    assert_sse(got["sse"], ref["sse"])
    assert_sse(got["f_opt"], ref["f_opt"])
    assert np.array_equal(got["degenerate"], ref["deg"])
    assert_centroids(got["centroids"].cpu().numpy(), ref["C"], ref["deg"], Xf, ref["labels"])
    assert_labels(got["labels"].cpu().numpy(), ref["labels"], Xf, ref["C"], ref["deg"])
    for key in ("samples", "replacements", "reseeded", "lloyd_iters", "n_d"):
        assert got["stats"][key] == ref["stats"][key], key
