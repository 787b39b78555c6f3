"""End-to-end Big-means parity (Alg. 1 + final assignment) against the oracle on
the same seeded input: sampled indices bit-exact, per-sample objectives, final
SSE and centroids to 1e-6 relative, integer counters exact."""
import json
import os

import numpy as np
import pytest
import torch

import oracle
from paper_2204_07485_amd import synth
from tests.parity import assert_centroids, assert_labels, assert_sse

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def _compare(X, got, ref, T, exact_counters=True):
    assert np.array_equal(got["sample_idx"].cpu().numpy(), ref["sample_idx"])
    sf_g, sf_r = got["sample_f"], ref["sample_f"]
    rel = np.abs(sf_g - sf_r) / sf_r
    first_bad = int(np.argmax(rel > 1e-6)) if (rel > 1e-6).any() else None
    assert first_bad is None, f"per-sample objective diverges first at sample {first_bad}: {rel[first_bad]:.3e}"
    assert_sse(got["sse"], ref["sse"])
    assert_sse(got["f_opt"], ref["f_opt"])
    assert np.array_equal(got["degenerate"], ref["deg"])
    assert_centroids(got["centroids"].cpu().numpy(), ref["C"], ref["deg"], X, ref["labels"])
    assert_labels(got["labels"].cpu().numpy(), ref["labels"], X, ref["C"], ref["deg"])
    if exact_counters:
        gs, rs = got["stats"], ref["stats"]
        assert gs["samples"] == rs["samples"] == T
        assert gs["replacements"] == rs["replacements"]
        assert gs["reseeded"] == rs["reseeded"]
        assert gs["lloyd_iters"] == rs["lloyd_iters"]
        assert gs["n_d"] == rs["n_d"]


def test_small_workload_matches_oracle():
    # 20,000 x 8, 10 isotropic Gaussians, k=10, s=2,000, 20 samples,
    # Lloyd until centroid shift < 1e-4 or 100 rounds
    from paper_2204_07485_amd import bigmeans
    W = synth.SMALL
    X = synth.make_small()
    print(f"fit small n={W.n} d={W.d} k={W.k} s={W.s} T={W.n_samples}", flush=True)
    got = bigmeans.bigmeans_fit(torch.from_numpy(X).cuda(), W.k, W.s, W.n_samples, W.seed,
                                sample_idx=True, max_iter=100, tol=1e-4,
                                stop_rule=bigmeans.BM_STOP_SHIFT)
    ref = oracle.bigmeans_fit(X, W.k, W.s, W.n_samples, W.seed, max_iter=100, tol=1e-4,
                              stop_rule=oracle.ORC_STOP_SHIFT, want_sample_idx=True)
    _compare(X, got, ref, W.n_samples)


@pytest.mark.parametrize("grid", [1, 5, 64])
def test_small_workload_any_grid(grid):
    from paper_2204_07485_amd import bigmeans
    X, _ = synth.gaussian_mixture(30_000, 5, 8, seed=21, sigma_range=(0.5, 2.0), weights="dirichlet")
    print(f"fit grid={grid}", flush=True)
    got = bigmeans.bigmeans_fit(torch.from_numpy(X).cuda(), 8, 3_001, 6, 99, sample_idx=True,
                                grid=grid, stop_rule=bigmeans.BM_STOP_REL_OBJ, max_iter=300)
    ref = oracle.bigmeans_fit(X, 8, 3_001, 6, 99, want_sample_idx=True,
                              stop_rule=oracle.ORC_STOP_REL_OBJ, max_iter=300)
    _compare(X, got, ref, 6)
    assert got["stats"]["grid"] == min(grid, 3_001)


def test_medium_workload_three_samples():
    # 1,000,000 x 16, 25 components, k=25, s=40,000, paper stop rule; 3 samples
    from paper_2204_07485_amd import bigmeans
    W = synth.MEDIUM
    X = synth.make_medium()
    T = 3
    print(f"fit medium T={T}", flush=True)
    got = bigmeans.bigmeans_fit(torch.from_numpy(X).cuda(), W.k, W.s, T, W.seed, sample_idx=True,
                                max_iter=300, tol=1e-4, stop_rule=bigmeans.BM_STOP_REL_OBJ)
    ref = oracle.bigmeans_fit(X, W.k, W.s, T, W.seed, max_iter=300, tol=1e-4,
                              stop_rule=oracle.ORC_STOP_REL_OBJ, want_sample_idx=True)
    _compare(X, got, ref, T)


def test_medium_workload_full_run_matches_stored_oracle():
    # the benchmark's workload and launch configuration, against the oracle's
    # result stored by tests/golden/make_golden.py
    from paper_2204_07485_amd import bigmeans
    with open(os.path.join(HERE, "golden", "medium_fit.json")) as fh:
        gold = json.load(fh)
    W = synth.MEDIUM
    X = synth.make_medium()
    got = bigmeans.bigmeans_fit(torch.from_numpy(X).cuda(), W.k, W.s, W.n_samples, W.seed,
                                max_iter=300, tol=1e-4, stop_rule=bigmeans.BM_STOP_REL_OBJ)
    print(f"medium full: gpu sse {got['sse']!r} oracle {gold['sse']!r}", flush=True)
    assert_sse(got["sse"], gold["sse"])
    assert_sse(got["f_opt"], gold["f_opt"])
    np.testing.assert_allclose(got["sample_f"], gold["sample_f"], rtol=1e-6)
    assert got["degenerate"].tolist() == gold["deg"]
    assert got["stats"]["replacements"] == gold["stats"]["replacements"]
    assert got["stats"]["lloyd_iters"] == gold["stats"]["lloyd_iters"]
    assert got["stats"]["n_d"] == gold["stats"]["n_d"]
    assert_centroids(got["centroids"].cpu().numpy(), np.array(gold["C"]), np.array(gold["deg"]))
    _assert_label_counts(got, gold, X)


def _assert_label_counts(got, gold, X):
    """Cluster sizes of the final pass equal the stored oracle's, up to the
    points that are near ties of the oracle's final centroids (each such point
    may move between two clusters)."""
    from tests.parity import near_tie_count
    C = np.array([[np.nan if v is None else v for v in row] for row in gold["C"]])
    deg = np.array(gold["deg"], np.uint8)
    lab = got["labels"].cpu().numpy()
    counts = np.bincount(lab[lab >= 0], minlength=len(deg))
    diff = int(np.abs(counts - np.array(gold["label_counts"])).sum())
    if diff:
        near = near_tie_count(X, C, deg)
        assert diff <= 2 * near, f"label counts differ by {diff}, near ties {near}"


@pytest.mark.parametrize("precision", ["fp32", "bf16_mfma"])
def test_bf16_workload_full_run_matches_stored_oracle(precision):
    # the full BF16 workload (5,000,000 x 128 stored as BF16, k=100, s=200,000,
    # 30 samples, paper stop rule) against the oracle's stored result
    # (tests/golden/make_golden.py bf16), with either final-pass arithmetic
    from paper_2204_07485_amd import bigmeans
    with open(os.path.join(HERE, "golden", "bf16_fit.json")) as fh:
        gold = json.load(fh)
    W = synth.BF16
    H = synth.make_bf16()
    prec = bigmeans.BM_PREC_BF16_MFMA if precision == "bf16_mfma" else bigmeans.BM_PREC_FP32
    print(f"bf16 full fit precision={precision}", flush=True)
    got = bigmeans.bigmeans_fit(torch.from_numpy(H.view(np.int16)).cuda(), W.k, W.s, W.n_samples,
                                W.seed, max_iter=300, tol=1e-4, stop_rule=bigmeans.BM_STOP_REL_OBJ,
                                precision=prec)
    print(f"bf16 full: gpu sse {got['sse']!r} oracle {gold['sse']!r}", flush=True)
    rel = np.abs(got["sample_f"] - np.array(gold["sample_f"])) / np.array(gold["sample_f"])
    first_bad = int(np.argmax(rel > 1e-6)) if (rel > 1e-6).any() else None
    assert first_bad is None, f"sample objective diverges first at sample {first_bad}"
    assert_sse(got["sse"], gold["sse"])
    assert_sse(got["f_opt"], gold["f_opt"])
    assert got["degenerate"].tolist() == gold["deg"]
    for key in ("replacements", "lloyd_iters", "n_d", "reseeded"):
        assert got["stats"][key] == gold["stats"][key], key
    Cg = np.array([[np.nan if v is None else v for v in row] for row in gold["C"]])
    assert_centroids(got["centroids"].cpu().numpy(), Cg, np.array(gold["deg"]))
    _assert_label_counts(got, gold, synth.bf16_bits_to_f32(H))


def test_resume_equals_uninterrupted():
    from paper_2204_07485_amd import bigmeans
    X, _ = synth.gaussian_mixture(50_000, 6, 12, seed=5, sigma_range=(0.5, 2.0), weights="dirichlet")
    Xd = torch.from_numpy(X).cuda()
    full = bigmeans.bigmeans_fit(Xd, 12, 4000, 9, 17)
    first = bigmeans.bigmeans_fit(Xd, 12, 4000, 4, 17, want_labels=False, want_sse=False)
    rest = bigmeans.bigmeans_fit(Xd, 12, 4000, 5, 17, t_start=4,
                                 state=(first["centroids"], first["degenerate"], first["f_opt"]))
    assert torch.equal(full["labels"], rest["labels"])
    assert np.array_equal(full["degenerate"], rest["degenerate"])
    assert full["sse"] == rest["sse"]
    assert full["f_opt"] == rest["f_opt"]
    assert np.array_equal(full["sample_f"], np.concatenate([first["sample_f"], rest["sample_f"]]))
    a = full["centroids"].cpu().numpy()
    b = rest["centroids"].cpu().numpy()
    assert np.array_equal(np.isnan(a), np.isnan(b)) and np.array_equal(a[~np.isnan(a)], b[~np.isnan(b)])


def test_deterministic_integer_outputs():
    from paper_2204_07485_amd import bigmeans
    X = synth.make_small()
    Xd = torch.from_numpy(X).cuda()
    a = bigmeans.bigmeans_fit(Xd, 10, 2000, 8, 3, sample_idx=True)
    b = bigmeans.bigmeans_fit(Xd, 10, 2000, 8, 3, sample_idx=True)
    assert torch.equal(a["sample_idx"], b["sample_idx"])
    assert torch.equal(a["labels"], b["labels"])
    assert a["stats"]["lloyd_iters"] == b["stats"]["lloyd_iters"]


def test_resample_compare_rule_matches_oracle():
    from paper_2204_07485_amd import bigmeans
    X, _ = synth.gaussian_mixture(40_000, 4, 6, seed=31, sigma_range=(0.5, 2.0))
    got = bigmeans.bigmeans_fit(torch.from_numpy(X).cuda(), 6, 1500, 10, 8, sample_idx=True,
                                compare_rule=bigmeans.BM_CMP_RESAMPLE)
    ref = oracle.bigmeans_fit(X, 6, 1500, 10, 8, want_sample_idx=True,
                              compare_rule=oracle.ORC_CMP_RESAMPLE)
    _compare(X, got, ref, 10)


def test_bf16_input_matches_oracle():
    from paper_2204_07485_amd import bigmeans
    X, _ = synth.gaussian_mixture(60_000, 32, 10, seed=13, sigma_range=(0.5, 2.0), outlier_frac=0.1)
    H = synth.to_bf16_bits(X)
    got = bigmeans.bigmeans_fit(torch.from_numpy(H.view(np.int16)).cuda(), 10, 5000, 4, 2,
                                sample_idx=True, stop_rule=bigmeans.BM_STOP_REL_OBJ, max_iter=300)
    ref = oracle.bigmeans_fit(H, 10, 5000, 4, 2, want_sample_idx=True,
                              stop_rule=oracle.ORC_STOP_REL_OBJ, max_iter=300)
    _compare(synth.bf16_bits_to_f32(H), got, ref, 4)


def test_k_equals_s_equals_n():
    from paper_2204_07485_amd import bigmeans
    X = np.arange(24, dtype=np.float32).reshape(12, 2)
    got = bigmeans.bigmeans_fit(torch.from_numpy(X).cuda(), 12, 12, 2, 1)
    assert got["sse"] == 0.0
    assert not got["degenerate"].any()


@pytest.mark.parametrize("mode", [1, 2])
def test_presampled_and_in_kernel_samples_agree(mode):
    # all samples drawn before the solver (automatic) vs. drawn by the solver
    # (presampling off, or a reported window miss): the same samples (Sec. 3.2
    # keys) and so the same fit
    from paper_2204_07485_amd import bigmeans
    W = synth.SMALL
    X = torch.from_numpy(synth.make_small()).cuda()
    kw = dict(sample_idx=True, max_iter=100, tol=1e-4, stop_rule=bigmeans.BM_STOP_SHIFT)
    ref = bigmeans.bigmeans_fit(X, W.k, W.s, W.n_samples, W.seed, **kw)
    prev = bigmeans.debug_presample(mode)
    try:
        got = bigmeans.bigmeans_fit(X, W.k, W.s, W.n_samples, W.seed, **kw)
    finally:
        bigmeans.debug_presample(prev)
    assert torch.equal(got["sample_idx"], ref["sample_idx"])
    assert np.array_equal(got["degenerate"], ref["degenerate"])
    np.testing.assert_allclose(got["sample_f"], ref["sample_f"], rtol=1e-9)
    assert_sse(got["sse"], ref["sse"])


@pytest.mark.parametrize("workload", ["small", "medium3", "bf16_mfma"])
def test_every_draw_with_row_order_sums(workload):
    # the row-order K-means++ draw (taken for draws near a running-sum
    # boundary) forced for every draw: in the persistent solver (FP32 fits)
    # and in the reseeding kernel (matrix-core fits) the fit must still equal
    # the oracle's, and every draw must have been counted as retaken
    from paper_2204_07485_amd import bigmeans
    print(f"fit with row-order draws: {workload}", flush=True)
    if workload == "small":
        W = synth.SMALL
        X = synth.make_small()
        args = (W.k, W.s, W.n_samples, W.seed)
        kw = dict(max_iter=100, tol=1e-4, stop_rule=bigmeans.BM_STOP_SHIFT)
        okw = dict(max_iter=100, tol=1e-4, stop_rule=oracle.ORC_STOP_SHIFT)
        Xg, Xo, Xf = torch.from_numpy(X).cuda(), X, X
    elif workload == "medium3":
        W = synth.MEDIUM
        X = synth.make_medium()
        args = (W.k, W.s, 3, W.seed)
        kw = dict(max_iter=300, tol=1e-4, stop_rule=bigmeans.BM_STOP_REL_OBJ)
        okw = dict(max_iter=300, tol=1e-4, stop_rule=oracle.ORC_STOP_REL_OBJ)
        Xg, Xo, Xf = torch.from_numpy(X).cuda(), X, X
    else:
        X, _ = synth.gaussian_mixture(60_000, 40, 12, seed=53, sigma_range=(0.5, 2.0), outlier_frac=0.1)
        H = synth.to_bf16_bits(X)
        args = (12, 6000, 5, 2)
        kw = dict(max_iter=300, stop_rule=bigmeans.BM_STOP_REL_OBJ, precision=bigmeans.BM_PREC_BF16_MFMA)
        okw = dict(max_iter=300, stop_rule=oracle.ORC_STOP_REL_OBJ)
        Xg, Xo, Xf = torch.from_numpy(H.view(np.int16)).cuda(), H, synth.bf16_bits_to_f32(H)
    prev = bigmeans.debug_exact_draws(1)
    try:
        got = bigmeans.bigmeans_fit(Xg, *args, sample_idx=True, **kw)
    finally:
        bigmeans.debug_exact_draws(prev)
    assert prev == 0
    ref = oracle.bigmeans_fit(Xo, *args, want_sample_idx=True, **okw)
    _compare(Xf, got, ref, args[2])
    # every reseed after the first placed centre draws n_local_trials targets
    assert got["stats"]["boundary_draws"] > 0
    assert got["stats"]["boundary_draws"] <= 3 * got["stats"]["reseeded"]
