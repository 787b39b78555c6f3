"""GPU parity of the modes beyond the sequential Big-means loop, each against
the oracle on the same seeded input:

- Forgy-style reinitialisation of degenerate centroids (Sec. 3.3);
- the time budget, the paper's stop condition (Sec. 5): a run stopped by its
  budget after m samples is exactly the run of m samples;
- the full-data K-means polish and "Big-means as initialiser" (Sec. 3.4);
- the collective parallel mode (Sec. 3.6, third scheme);
- the sample-size rule of thumb (Sec. 5).
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2204_07485_amd import synth
from tests.parity import LABEL_TIE_REL, assert_centroids, assert_labels, assert_sse, top2_gap

pytestmark = pytest.mark.gpu


def _first_bad(got, ref, rel=1e-6):
    r = np.abs(np.asarray(got) - np.asarray(ref)) / np.abs(np.asarray(ref))
    return int(np.argmax(r > rel)) if (r > rel).any() else None


def _fit_compare(X, got, ref, T):
    assert np.array_equal(got["sample_idx"].cpu().numpy(), ref["sample_idx"])
    bad = _first_bad(got["sample_f"], ref["sample_f"])
    assert bad is None, f"per-sample objective diverges first at sample {bad}"
    assert_sse(got["sse"], ref["sse"])
    assert_sse(got["f_opt"], ref["f_opt"])
    assert np.array_equal(got["degenerate"], ref["deg"])
    assert_centroids(got["centroids"].cpu().numpy(), ref["C"], ref["deg"], X, ref["labels"])
    assert_labels(got["labels"].cpu().numpy(), ref["labels"], X, ref["C"], ref["deg"])
    for key in ("samples", "replacements", "reseeded", "lloyd_iters", "n_d"):
        assert got["stats"][key] == ref["stats"][key], key
    assert got["stats"]["samples"] == T


# ------------------------------------------------------------------- Forgy

@pytest.mark.parametrize("presample", [0, 1])
def test_forgy_initialisation_matches_oracle(presample):
    from paper_2204_07485_amd import bigmeans
    W = synth.SMALL
    X = synth.make_small()
    prev = bigmeans.debug_presample(presample)
    try:
        got = bigmeans.bigmeans_fit(torch.from_numpy(X).cuda(), W.k, W.s, W.n_samples, W.seed,
                                    sample_idx=True, init_method=bigmeans.BM_INIT_FORGY)
    finally:
        bigmeans.debug_presample(prev)
    ref = oracle.bigmeans_fit(X, W.k, W.s, W.n_samples, W.seed, want_sample_idx=True,
                              init_method=oracle.ORC_INIT_FORGY)
    _fit_compare(X, got, ref, W.n_samples)


def test_forgy_on_the_medium_workload_three_samples():
    from paper_2204_07485_amd import bigmeans
    W = synth.MEDIUM
    X = synth.make_medium()
    kw = dict(max_iter=300, tol=1e-4)
    got = bigmeans.bigmeans_fit(torch.from_numpy(X).cuda(), W.k, W.s, 3, W.seed, sample_idx=True,
                                stop_rule=bigmeans.BM_STOP_REL_OBJ,
                                init_method=bigmeans.BM_INIT_FORGY, **kw)
    ref = oracle.bigmeans_fit(X, W.k, W.s, 3, W.seed, want_sample_idx=True,
                              stop_rule=oracle.ORC_STOP_REL_OBJ,
                              init_method=oracle.ORC_INIT_FORGY, **kw)
    _fit_compare(X, got, ref, 3)


# ------------------------------------------------------------- time budget

def test_time_budget_stops_at_a_sample_boundary():
    from paper_2204_07485_amd import bigmeans
    X, _ = synth.gaussian_mixture(200_000, 16, 12, seed=41, sigma_range=(0.5, 2.0),
                                  weights="dirichlet")
    Xd = torch.from_numpy(X).cuda()
    kw = dict(max_iter=300, tol=1e-4, stop_rule=bigmeans.BM_STOP_REL_OBJ)
    cap = 100_000
    got = bigmeans.bigmeans_fit(Xd, 12, 20_000, cap, 7, time_budget_ms=25.0, sample_idx=False,
                                **kw)
    m = got["stats"]["samples"]
    print(f"budget 25 ms: {m} samples, solver {got['stats']['ms_solver']:.2f} ms", flush=True)
    assert 1 <= m < cap
    assert got["stats"]["ms_solver"] >= 25.0 * 0.98
    # processing m samples under the budget is the run of m samples
    # (FP64 cluster sums are added atomically, so only rounding may differ)
    plain = bigmeans.bigmeans_fit(Xd, 12, 20_000, m, 7, **kw)
    np.testing.assert_allclose(got["sample_f"][:m], plain["sample_f"], rtol=1e-9)
    assert_sse(got["sse"], plain["sse"], rel=1e-9)
    assert np.array_equal(got["degenerate"], plain["degenerate"])
    assert got["stats"]["replacements"] == plain["stats"]["replacements"]
    assert_labels(got["labels"].cpu().numpy(), plain["labels"].cpu().numpy(), X,
                  plain["centroids"].cpu().numpy(), plain["degenerate"])
    mo = min(m, 12)
    ref = oracle.bigmeans_fit(X, 12, 20_000, mo, 7, stop_rule=oracle.ORC_STOP_REL_OBJ,
                              max_iter=300, tol=1e-4)
    bad = _first_bad(got["sample_f"][:mo], ref["sample_f"])
    assert bad is None, f"per-sample objective diverges first at sample {bad}"


def test_time_budget_larger_than_the_run():
    from paper_2204_07485_amd import bigmeans
    X = synth.make_small()
    W = synth.SMALL
    Xd = torch.from_numpy(X).cuda()
    got = bigmeans.bigmeans_fit(Xd, W.k, W.s, W.n_samples, W.seed, time_budget_ms=60_000.0)
    ref = bigmeans.bigmeans_fit(Xd, W.k, W.s, W.n_samples, W.seed)
    assert got["stats"]["samples"] == W.n_samples
    np.testing.assert_allclose(got["sample_f"], ref["sample_f"], rtol=1e-9)
    assert_sse(got["sse"], ref["sse"], rel=1e-9)


# ------------------------------------------------------ polish / initialiser

def _separated(n, d, comps, seed):
    return synth.gaussian_mixture(n, d, comps, seed, sigma_range=(0.3, 0.6), weights="dirichlet")[0]


def test_initialiser_mode_skips_the_final_pass():
    from paper_2204_07485_amd import bigmeans
    X = _separated(150_000, 16, 20, seed=42)
    Xd = torch.from_numpy(X).cuda()
    full = bigmeans.bigmeans_fit(Xd, 20, 10_000, 8, 3)
    init = bigmeans.bigmeans_fit(Xd, 20, 10_000, 8, 3, want_labels=False, want_sse=False)
    assert init["stats"]["ms_final"] == 0.0 and init["labels"] is None  # no final pass ran
    assert torch.equal(full["centroids"].isnan(), init["centroids"].isnan())
    assert torch.equal(torch.nan_to_num(full["centroids"]), torch.nan_to_num(init["centroids"]))
    assert init["f_opt"] == full["f_opt"]


@pytest.mark.parametrize("rule,max_iter", [(1, 300), (0, 100), (0, 2)])
def test_polish_is_kmeans_on_all_of_x(rule, max_iter):
    # Sec. 3.4: K-means over the whole dataset from the Big-means centroids
    from paper_2204_07485_amd import bigmeans
    X = _separated(150_000, 16, 20, seed=43)
    Xd = torch.from_numpy(X).cuda()
    kw = dict(max_iter=max_iter, tol=1e-4, stop_rule=rule)
    init = bigmeans.bigmeans_fit(Xd, 20, 5_000, 6, 4, want_labels=False, want_sse=False, **kw)
    pol = bigmeans.bigmeans_fit(Xd, 20, 5_000, 6, 4, final_mode=bigmeans.BM_FINAL_POLISH, **kw)
    C0 = init["centroids"].cpu().numpy().astype(np.float64)
    deg0 = init["degenerate"]
    rC, rdeg, rlab, rf, rp, _ = oracle.lloyd(X, C0, deg0, **kw)
    # near ties along the oracle's path decide how strict the comparison is
    C, deg, gap = C0, deg0.copy(), np.inf
    for _ in range(min(rp, 30)):
        gap = min(gap, float(top2_gap(X, C.astype(np.float32), deg).min()))
        nC, ndeg, _, _, _, _ = oracle.lloyd(X, C.astype(np.float32), deg, max_iter=1, tol=0.0)
        if np.allclose(nC, C, equal_nan=True, rtol=0, atol=0):
            break
        C, deg = nC, ndeg
    print(f"polish rule={rule} max_iter={max_iter}: passes gpu {pol['stats']['final_passes']} "
          f"oracle {rp}, min gap {gap:.2e}", flush=True)
    lab = pol["labels"].cpu().numpy()
    gC = pol["centroids"].cpu().numpy()
    if gap >= LABEL_TIE_REL:
        assert pol["stats"]["final_passes"] == rp
        assert np.array_equal(pol["degenerate"], rdeg)
        assert_sse(pol["sse"], rf)
        assert_centroids(gC, rC, rdeg, X, rlab)
        assert_labels(lab, rlab, X, rC, rdeg)
    # at any rate the result is that of its own centroids
    with oracle.threaded():
        olab, _, of = oracle.assign(X, gC, pol["degenerate"])
    assert_sse(pol["sse"], of)
    assert_labels(lab, olab, X, gC, pol["degenerate"])
    assert pol["sse"] <= of * (1 + 1e-6)


def test_polish_rejects_bf16_points():
    from paper_2204_07485_amd import bigmeans
    X = torch.zeros((100, 4), dtype=torch.bfloat16, device="cuda")
    with pytest.raises(bigmeans.BigmeansError) as e:
        bigmeans.bigmeans_fit(X, 2, 10, 1, 1, final_mode=bigmeans.BM_FINAL_POLISH)
    assert e.value.code == bigmeans.BM_ENOTSUP


# -------------------------------------------------------------- collective

@pytest.mark.parametrize("W,R,init", [(4, 5, 0), (1, 6, 0), (3, 4, 1)])
def test_collective_matches_oracle(W, R, init):
    from paper_2204_07485_amd import bigmeans
    S = synth.SMALL
    X = synth.make_small()
    kw = dict(max_iter=100, tol=1e-4)
    got = bigmeans.bigmeans_fit_collective(torch.from_numpy(X).cuda(), S.k, S.s, W, R, S.seed,
                                           stop_rule=bigmeans.BM_STOP_SHIFT, init_method=init, **kw)
    ref = oracle.bigmeans_collective(X, S.k, S.s, W, R, S.seed, stop_rule=oracle.ORC_STOP_SHIFT,
                                     init_method=init, **kw)
    print(f"collective W={W} R={R}: gpu sse {got['sse']!r} oracle {ref['sse']!r}", flush=True)
    bad = _first_bad(got["worker_f"].ravel(), ref["worker_f"].ravel())
    assert bad is None, f"worker objective diverges first at (round, worker) {divmod(bad, W)}"
    assert_sse(got["sse"], ref["sse"])
    assert_sse(got["f_opt"], ref["f_opt"])
    assert np.array_equal(got["degenerate"], ref["deg"])
    assert_centroids(got["centroids"].cpu().numpy(), ref["C"], ref["deg"], X, ref["labels"])
    assert_labels(got["labels"].cpu().numpy(), ref["labels"], X, ref["C"], ref["deg"])
    for key in ("samples", "replacements", "reseeded", "lloyd_iters"):
        assert got["stats"][key] == ref["stats"][key], key


def test_collective_one_worker_equals_bigmeans_fit():
    from paper_2204_07485_amd import bigmeans
    S = synth.SMALL
    Xd = torch.from_numpy(synth.make_small()).cuda()
    a = bigmeans.bigmeans_fit_collective(Xd, S.k, S.s, 1, S.n_samples, S.seed)
    b = bigmeans.bigmeans_fit(Xd, S.k, S.s, S.n_samples, S.seed)
    np.testing.assert_allclose(a["worker_f"][:, 0], b["sample_f"], rtol=1e-6)
    assert_sse(a["sse"], b["sse"])
    assert a["stats"]["replacements"] == b["stats"]["replacements"]


def test_collective_rejects_resample_rule():
    from paper_2204_07485_amd import bigmeans
    Xd = torch.from_numpy(synth.make_small()).cuda()
    with pytest.raises(bigmeans.BigmeansError) as e:
        bigmeans.bigmeans_fit_collective(Xd, 4, 500, 2, 2, 1, compare_rule=bigmeans.BM_CMP_RESAMPLE)
    assert e.value.code == bigmeans.BM_ENOTSUP


# -------------------------------------------------------------- sample size

def test_sample_size_sweep_matches_oracle():
    from paper_2204_07485_amd import bigmeans
    rng = np.random.default_rng(16)
    mu = rng.uniform(-20, 20, size=(25, 2))
    lab = rng.integers(0, 25, size=8000)
    X = (mu[lab] + 0.5 * rng.normal(size=(8000, 2))).astype(np.float32)
    got = bigmeans.sample_size_sweep(torch.from_numpy(X).cuda(), 25, 30, 8000, 3, 3)
    best, tried = oracle.sample_size_sweep(X, 25, 30, 8000, 3, seed=3)
    print(f"sweep gpu {got['tried']} oracle {tried}", flush=True)
    assert [s for s, _ in got["tried"]] == [s for s, _ in tried]
    for (_, a), (_, b) in zip(got["tried"], tried):
        assert_sse(a, b)
    assert got["s_best"] == best
    assert_sse(got["sse"], dict(tried)[best])


def test_collective_medium_workload_matches_stored_oracle():
    # the benchmark's collective configuration: the medium workload with 8
    # workers x 7 rounds, against tests/golden/medium_collective.json
    import json
    import os
    from paper_2204_07485_amd import bigmeans
    with open(os.path.join(os.path.dirname(__file__), "golden", "medium_collective.json")) as fh:
        gold = json.load(fh)
    W = synth.MEDIUM
    X = synth.make_medium()
    got = bigmeans.bigmeans_fit_collective(torch.from_numpy(X).cuda(), W.k, W.s, gold["workers"],
                                           gold["rounds"], W.seed, max_iter=300, tol=1e-4,
                                           stop_rule=bigmeans.BM_STOP_REL_OBJ)
    print(f"collective medium: gpu sse {got['sse']!r} oracle {gold['sse']!r}", flush=True)
    bad = _first_bad(got["worker_f"].ravel(), np.array(gold["worker_f"]).ravel())
    assert bad is None, f"worker objective diverges first at (round, worker) {divmod(bad, 8)}"
    assert_sse(got["sse"], gold["sse"])
    assert_sse(got["f_opt"], gold["f_opt"])
    assert got["degenerate"].tolist() == gold["deg"]
    for key in ("replacements", "reseeded", "lloyd_iters"):
        assert got["stats"][key] == gold["stats"][key], key
    Cg = np.array([[np.nan if v is None else v for v in row] for row in gold["C"]])
    assert_centroids(got["centroids"].cpu().numpy(), Cg, np.array(gold["deg"]))
