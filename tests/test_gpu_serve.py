"""GPU tests of the serving context (bm_ctx): a job run in a mix of
concurrent jobs gives the result it gives alone (same samples, so the same
per-sample objectives, degenerate flags and final objective, to the parity
tolerance), admission keeps the scratch held within the budget, and
cancellation, timeouts and failures are reported per job while the context
keeps serving."""
import time

import numpy as np
import pytest
import torch

from paper_2204_07485_amd import synth
from tests.parity import assert_sse

pytestmark = pytest.mark.gpu

KW = dict(max_iter=300, tol=1e-4, stop_rule=1, n_local_trials=3)


def _jobs(count, seed=5, n_range=(1e4, 2e5)):
    out = []
    for job in synth.serve_jobs(count, seed=seed, n_range=n_range):
        X = torch.from_numpy(synth.serve_job_data(job)).cuda()
        out.append((job, X))
    return out


def test_mix_equals_alone():
    from paper_2204_07485_amd import bigmeans
    jobs = _jobs(12)
    with bigmeans.Server(slots=4) as srv:
        ids = [srv.submit(X, j["k"], j["s"], j["n_samples"], j["seed"], **KW) for j, X in jobs]
        res = [srv.result(i) for i in ids]
        grid = srv.info()["grid_per_job"]
        info = srv.info()
    assert info["completed"] == len(jobs) and info["failed"] == 0
    overlap = 0
    for a in range(len(res)):
        for b in range(a + 1, len(res)):
            if res[a]["t_start_ms"] < res[b]["t_end_ms"] and res[b]["t_start_ms"] < res[a]["t_end_ms"]:
                overlap += 1
    assert overlap > 0, "no two jobs ran at the same time"
    for (j, X), r in zip(jobs, res):
        print(f"job {j['id']}: n={j['n']} d={j['d']} k={j['k']}", flush=True)
        alone = bigmeans.bigmeans_fit(X, j["k"], j["s"], j["n_samples"], j["seed"], grid=grid, **KW)
        assert np.array_equal(r["degenerate"], alone["degenerate"])
        np.testing.assert_allclose(r["sample_f"], alone["sample_f"], rtol=1e-6)
        assert_sse(r["sse"], alone["sse"])
        assert r["stats"]["samples"] == alone["stats"]["samples"]


def test_budget_bounds_the_scratch_held():
    from paper_2204_07485_amd import bigmeans
    jobs = _jobs(8, seed=6)
    # a budget that holds the largest job but not two of the largest
    with bigmeans.Server(slots=4, hbm_budget=1 << 40) as srv:
        ids = [srv.submit(X, j["k"], j["s"], j["n_samples"], j["seed"], **KW) for j, X in jobs]
        big = max(srv.poll(i).footprint for i in ids)
        for i in ids:
            srv.result(i)
    budget = int(big * 1.5)
    with bigmeans.Server(slots=4, hbm_budget=budget) as srv:
        ids = [srv.submit(X, j["k"], j["s"], j["n_samples"], j["seed"], **KW) for j, X in jobs]
        res = [srv.result(i) for i in ids]
        info = srv.info()
    assert info["completed"] == len(jobs)
    assert info["peak_reserved_bytes"] <= budget
    # jobs started in submission order
    starts = [r["t_start_ms"] for r in res]
    assert starts == sorted(starts)


def test_cancel_timeout_and_oversized_job():
    from paper_2204_07485_amd import bigmeans
    jobs = _jobs(5, seed=7)
    with bigmeans.Server(slots=1) as srv:
        ids = [srv.submit(X, j["k"], j["s"], j["n_samples"], j["seed"], **KW) for j, X in jobs]
        last = ids[-1]
        with pytest.raises(bigmeans.BigmeansError) as e:
            srv.wait(last, timeout_ms=0)
        assert e.value.code == bigmeans.BM_ETIMEDOUT
        srv.cancel(last)
        assert srv.poll(last).state == bigmeans.BM_JOB_CANCELLED
        with pytest.raises(bigmeans.BigmeansError) as e:
            srv.result(last)
        assert e.value.code == bigmeans.BM_ECANCELLED
        for i in ids[:-1]:
            assert srv.result(i)["sse"] > 0
        with pytest.raises(bigmeans.BigmeansError):
            srv.cancel(ids[0])  # finished: no longer cancellable
    with bigmeans.Server(slots=2, hbm_budget=2 << 20) as srv:
        j, X = jobs[0]
        with pytest.raises(bigmeans.BigmeansError) as e:
            srv.submit(X, j["k"], j["s"], j["n_samples"], j["seed"], **KW)
        assert e.value.code == bigmeans.BM_ENOMEM


def test_failed_job_is_reported_and_serving_continues():
    from paper_2204_07485_amd import bigmeans
    jobs = _jobs(3, seed=8)
    with bigmeans.Server(slots=2) as srv:
        j, X = jobs[0]
        bad = srv.submit(X, j["k"], j["s"], j["n_samples"], j["seed"], spin_limit=1, **KW)
        good = [srv.submit(X2, j2["k"], j2["s"], j2["n_samples"], j2["seed"], **KW)
                for j2, X2 in jobs[1:]]
        info = srv.wait(bad)
        assert info.state == bigmeans.BM_JOB_FAILED
        assert info.result == bigmeans.BM_EDEVICE and info.error
        for i in good:
            assert srv.result(i)["sse"] > 0
        assert srv.info()["failed"] == 1


def test_rounds_mode_matches_whole_fits():
    # continuous batching (BM_SERVE_ROUNDS): the jobs' Lloyd rounds share
    # batched launches; every job must still give what bigmeans_fit gives it
    # alone (same samples and reseeds; objectives to rounding, since the
    # batched kernels sum in another order)
    from paper_2204_07485_amd import bigmeans
    jobs = _jobs(12, seed=8)
    with bigmeans.Server(slots=6, mode=bigmeans.BM_SERVE_ROUNDS) as srv:
        ids = [srv.submit(X, j["k"], j["s"], j["n_samples"], j["seed"], **KW) for j, X in jobs]
        res = [srv.result(i) for i in ids]
        info = srv.info()
    assert info["completed"] == len(jobs) and info["failed"] == 0
    overlap = 0
    for a in range(len(res)):
        for b in range(a + 1, len(res)):
            if res[a]["t_start_ms"] < res[b]["t_end_ms"] and res[b]["t_start_ms"] < res[a]["t_end_ms"]:
                overlap += 1
    assert overlap > 0, "no two jobs were in flight together"
    for (j, X), r in zip(jobs, res):
        print(f"job {j['id']}: n={j['n']} d={j['d']} k={j['k']} s={j['s']}", flush=True)
        alone = bigmeans.bigmeans_fit(X, j["k"], j["s"], j["n_samples"], j["seed"], **KW)
        assert np.array_equal(r["degenerate"], alone["degenerate"])
        np.testing.assert_allclose(r["sample_f"], alone["sample_f"], rtol=1e-6)
        assert_sse(r["sse"], alone["sse"])
        assert r["stats"]["samples"] == alone["stats"]["samples"] == j["n_samples"]
        assert r["stats"]["replacements"] == alone["stats"]["replacements"]
        assert abs(r["stats"]["lloyd_iters"] - alone["stats"]["lloyd_iters"]) <= \
            0.02 * alone["stats"]["lloyd_iters"] + 2
        assert r["stats"]["reseeded"] == alone["stats"]["reseeded"]
        np.testing.assert_allclose(r["centroids"].cpu().numpy(), alone["centroids"].cpu().numpy(),
                                   rtol=1e-5, atol=1e-5)


def test_rounds_mode_bf16_input_and_labels():
    from paper_2204_07485_amd import bigmeans
    X32, _ = synth.gaussian_mixture(60_000, 32, 12, seed=31, sigma_range=(0.5, 2.0))
    X = torch.from_numpy(X32).cuda().to(torch.bfloat16)
    specs = ((12, 8_000, 6, 77), (7, 5_000, 4, 78))
    with bigmeans.Server(slots=2, mode=bigmeans.BM_SERVE_ROUNDS) as srv:
        ids = [srv.submit(X, k, s, T, seed, want_labels=True, **KW) for k, s, T, seed in specs]
        res = [srv.result(i) for i in ids]
    for r, (k, s, T, seed) in zip(res, specs):
        alone = bigmeans.bigmeans_fit(X, k, s, T, seed, **KW)
        assert_sse(r["sse"], alone["sse"])
        assert np.array_equal(r["degenerate"], alone["degenerate"])
        same = (r["labels"].cpu().numpy() == alone["labels"].cpu().numpy()).mean()
        assert same > 0.9999


def test_rounds_mode_rejects_what_it_cannot_batch():
    from paper_2204_07485_amd import bigmeans
    (j, X), = _jobs(1, seed=9)
    with bigmeans.Server(slots=2, mode=bigmeans.BM_SERVE_ROUNDS, round_max_k=8,
                         round_max_s=4_000) as srv:
        with pytest.raises(bigmeans.BigmeansError) as e:
            srv.submit(X, 9, 2_000, 3, 1, **KW)
        assert e.value.code == bigmeans.BM_ENOTSUP
        with pytest.raises(bigmeans.BigmeansError) as e:
            srv.submit(X, 4, 5_000, 3, 1, **KW)
        assert e.value.code == bigmeans.BM_ENOTSUP
        with pytest.raises(bigmeans.BigmeansError) as e:
            srv.submit(X, 4, 2_000, 3, 1, **dict(KW, compare_rule=bigmeans.BM_CMP_RESAMPLE))
        assert e.value.code == bigmeans.BM_ENOTSUP
        jid = srv.submit(X, 4, 2_000, 3, 1, **KW)
        r = srv.result(jid)
        alone = bigmeans.bigmeans_fit(X, 4, 2_000, 3, 1, **KW)
        assert_sse(r["sse"], alone["sse"])


def test_rounds_mode_reuses_slots_across_ticks():
    # more jobs than slots, equal sample sizes, arriving one by one: a freed
    # slot is taken by a later job after other rounds have run without it
    from paper_2204_07485_amd import bigmeans
    X, _ = synth.gaussian_mixture(40_000, 8, 6, seed=41, sigma_range=(0.5, 2.0))
    X = torch.from_numpy(X).cuda()
    specs = [(6, 4_000, 3 + (i % 3), 100 + i) for i in range(9)]
    with bigmeans.Server(slots=2, mode=bigmeans.BM_SERVE_ROUNDS) as srv:
        ids = []
        for k, s, T, seed in specs:
            ids.append(srv.submit(X, k, s, T, seed, **KW))
            time.sleep(0.003)
        res = [srv.result(i) for i in ids]
    for r, (k, s, T, seed) in zip(res, specs):
        alone = bigmeans.bigmeans_fit(X, k, s, T, seed, **KW)
        assert np.array_equal(r["degenerate"], alone["degenerate"])
        np.testing.assert_allclose(r["sample_f"], alone["sample_f"], rtol=1e-6)
        assert_sse(r["sse"], alone["sse"])


@pytest.mark.parametrize("mode", ["fits", "rounds"])
def test_served_jobs_match_oracle(mode):
    # served jobs (in a mix, several in flight) against the oracle's
    # Big-means on the same X and seed (Alg. 1 + final pass): per-sample
    # objectives, final objective and centroids to 1e-6, flags and
    # replacement/reseed counts exactly
    import oracle
    from paper_2204_07485_amd import bigmeans
    from tests.parity import assert_centroids
    jobs = [(j, X) for j, X in _jobs(10, seed=12, n_range=(1e4, 3e4)) if j["d"] <= 32][:5]
    m = bigmeans.BM_SERVE_ROUNDS if mode == "rounds" else bigmeans.BM_SERVE_FITS
    with bigmeans.Server(slots=3, mode=m) as srv:
        ids = [srv.submit(X, j["k"], j["s"], j["n_samples"], j["seed"], want_labels=True, **KW)
               for j, X in jobs]
        res = [srv.result(i) for i in ids]
    assert len(res) >= 3
    for (j, X), r in zip(jobs, res):
        print(f"{mode} job {j['id']}: n={j['n']} d={j['d']} k={j['k']} s={j['s']}", flush=True)
        Xh = X.cpu().numpy()
        with oracle.threaded():
            ref = oracle.bigmeans_fit(Xh, j["k"], j["s"], j["n_samples"], j["seed"],
                                      max_iter=KW["max_iter"], tol=KW["tol"],
                                      stop_rule=oracle.ORC_STOP_REL_OBJ,
                                      n_local_trials=KW["n_local_trials"])
        rel = np.abs(r["sample_f"] - ref["sample_f"]) / ref["sample_f"]
        first_bad = int(np.argmax(rel > 1e-6)) if (rel > 1e-6).any() else None
        assert first_bad is None, f"sample objective diverges first at sample {first_bad}"
        assert_sse(r["sse"], ref["sse"])
        assert np.array_equal(r["degenerate"], ref["deg"])
        assert r["stats"]["replacements"] == ref["stats"]["replacements"]
        assert r["stats"]["reseeded"] == ref["stats"]["reseeded"]
        assert_centroids(r["centroids"].cpu().numpy(), ref["C"], ref["deg"], Xh, ref["labels"])
        from tests.parity import assert_labels
        assert_labels(r["labels"].cpu().numpy(), ref["labels"], Xh, ref["C"], ref["deg"])
