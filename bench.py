"""Benchmark: Big-means time-to-oracle-SSE on one MI355X.

One step = one bigmeans_fit (Alg. 1: 50 samples of sampling, K-means++
reseeding, Lloyd and keep-the-best, then the final assignment of all points)
on the medium workload: 1,000,000 x 16 FP32 points from a 25-component
Gaussian mixture, k=25, s=40,000, seed 2, the paper's stop rule (relative
objective decrease <= 1e-4 or 300 rounds) and three K-means++ candidates.
X is resident in HBM before timing starts.  The final objective of every
timed fit is checked against the CPU oracle's stored objective (1e-6
relative); value is the mean wall time per fit.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
"""
import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# FP32 direct differences take two VALU instructions (subtract, FMA) per
# coordinate: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz x 2 FLOP / 2 instructions
FP32_DD_PEAK_TFLOPS = 256 * 4 * 16 * 2.4e9 * 2 / 2 / 1e12
FP32_MFMA_PEAK_TFLOPS = 157.3  # dense FP32 matrix (MI355X)
COUNTERS = os.path.join(ROOT, "profiles", "solver_medium_hbm_counters.md")


# the sources that define the profiled kernels (the persistent solver and the
# FP32 final pass) and how they are launched
PROFILED_SOURCES = ("bm_api.hip", "bm_solver.hip", "bm_assign.hip", "bm_assign_mfma32.hip",
                    "bm_device.h", "bm_internal.h", "bm_rng.h")


def source_hash():
    """Hash of the sources of the profiled kernels, to tell whether stored
    profiler byte counts still describe the kernels being timed."""
    import hashlib
    h = hashlib.sha256()
    files = [os.path.join(ROOT, "paper_2204_07485_amd", "csrc", f) for f in PROFILED_SOURCES]
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    summary, or None when the kernels changed since it was taken."""
    if not os.path.exists(COUNTERS):
        return None, None
    vals = {}
    with open(COUNTERS) as fh:
        for line in fh:
            if ":" in line and line.split(":")[0] in ("source-hash", "traffic_mb_solver",
                                                       "traffic_mb_final"):
                key, val = line.split(":", 1)
                vals[key.strip()] = val.strip()
    if vals.get("source-hash") != source_hash():
        return None, None
    return float(vals["traffic_mb_solver"]) * 1e6, float(vals["traffic_mb_final"]) * 1e6


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving stream")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-solves workload")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the BF16 workload's mixed-precision (MFMA) comparison")
    ap.add_argument("--no-final", action="store_true",
                    help="skip the cache-flushed final-pass timings")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the collective-mode and sample-size-sweep section (for profiling the headline)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after timing, run a plain 1 GiB device copy three times (a known "
                         "amount of HBM traffic for scaling profiler byte counters)")
    return ap.parse_args()


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(X, W):
    """The oracle as it stands, in its OpenMP build (per-point loops on all
    host cores, every sum in index order, results bit-identical to the
    single-threaded build), timed on the whole fit: all samples plus the
    final assignment pass."""
    import oracle
    with oracle.threaded():
        threads = oracle.threads()
        t0 = time.perf_counter()
        r = oracle.bigmeans_fit(X, W.k, W.s, W.n_samples, W.seed, max_iter=300, tol=1e-4,
                                stop_rule=oracle.ORC_STOP_REL_OBJ, want_labels=True, want_sse=True)
        secs = time.perf_counter() - t0
    return {"value": secs * 1e3, "unit": "ms", "cores": threads, "kind": "oracle",
            "sample": f"the whole fit ({W.n_samples} samples + final pass), OpenMP oracle build on "
                      f"{threads} threads; host: {os.cpu_count()} logical CPUs, {cpu_model()}",
            "oracle_sse": r["sse"]}


def flush_mall(buf):
    """Read a buffer larger than the 256 MB last-level cache so the next
    kernel finds none of its input there."""
    import torch
    buf.add_(1.0)
    torch.cuda.synchronize()


def mixed_precision(reps=5):
    """The BF16 workload (5,000,000 x 128 BF16, 100 components + 10% outliers,
    k=100, s=200,000, 30 samples, seed 4): one full fit per distance
    arithmetic, each checked against the oracle's stored result, then the final
    assignment pass alone timed with HIP events for both forms on the fit's
    centroids."""
    import numpy as np
    import torch

    from paper_2204_07485_amd import bigmeans, synth
    W = synth.BF16
    with open(os.path.join(ROOT, "tests", "golden", "bf16_fit.json")) as fh:
        gold = json.load(fh)
    H = synth.make_bf16()
    Hd = torch.from_numpy(H.view(np.int16)).to("cuda:0")
    del H
    kw = dict(max_iter=300, tol=1e-4, stop_rule=bigmeans.BM_STOP_REL_OBJ, n_local_trials=3)
    fits = {}
    for name, prec in (("fp32", bigmeans.BM_PREC_FP32), ("bf16_mfma", bigmeans.BM_PREC_BF16_MFMA)):
        bigmeans.bigmeans_fit(Hd, W.k, W.s, 2, W.seed, precision=prec, **kw)  # warm-up
        best = None
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = bigmeans.bigmeans_fit(Hd, W.k, W.s, W.n_samples, W.seed, precision=prec, **kw)
            ms = (time.perf_counter() - t0) * 1e3
            best = (r, ms) if best is None or ms < best[1] else best
        fits[name] = best
    C, deg = fits["bf16_mfma"][0]["centroids"], fits["bf16_mfma"][0]["degenerate"]
    ms = {}
    out = {}
    for name, prec in (("fp32", bigmeans.BM_PREC_FP32), ("bf16_mfma", bigmeans.BM_PREC_BF16_MFMA)):
        vals = []
        for _ in range(reps):
            lab, _, sse = bigmeans.kmeans_assign(Hd, C, deg, precision=prec)
            vals.append(bigmeans.last_assign_ms())
        ms[name] = statistics.median(vals)
        out[name] = (lab.cpu().numpy(), sse, bigmeans.last_rechecked() if prec else 0)
    n, d, k = W.n, W.d, W.k
    algo_bytes = n * d * 2 + n * 4
    kp = 16 * ((k + 15) // 16)
    gbs = algo_bytes / (ms["bf16_mfma"] * 1e-3) / 1e9
    rel = {name: abs(v[0]["sse"] - gold["sse"]) / gold["sse"] for name, v in fits.items()}
    return {
        "workload": "bf16: 5,000,000 x 128 BF16 Gaussian mixture (100 components, sigma "
                    "U[0.5,2], 10% uniform outliers), k=100, s=200,000, 30 samples, seed 4",
        "fit_ms": {k_: v[1] for k_, v in fits.items()},
        "time_to_oracle_sse_ms": {k_: (v[1] if rel[k_] <= 1e-6 else None) for k_, v in fits.items()},
        "fit_sse": {k_: v[0]["sse"] for k_, v in fits.items()},
        "oracle_sse": gold["sse"],
        "fit_sse_rel_err": rel,
        "fit_ms_solver": {k_: v[0]["stats"]["ms_solver"] for k_, v in fits.items()},
        "fit_ms_final": {k_: v[0]["stats"]["ms_final"] for k_, v in fits.items()},
        "final_pass_ms": ms,
        "final_pass_speedup": ms["fp32"] / ms["bf16_mfma"],
        "labels_equal": bool((out["fp32"][0] == out["bf16_mfma"][0]).all()),
        "sse_rel_diff": abs(out["fp32"][1] - out["bf16_mfma"][1]) / out["fp32"][1],
        "rechecked": int(out["bf16_mfma"][2]),
        "roofline": {"bound": "hbm", "kernel": "assign_mfma_kernel<4,true>", "achieved": gbs,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
                     "traffic": None, "algorithmic_bytes": algo_bytes,
                     "mfma_tflops": 2 * 2 * n * kp * d / (ms["bf16_mfma"] * 1e-3) / 1e12,
                     "fp32_path_tflops": 2 * n * k * d / (ms["fp32"] * 1e-3) / 1e12},
    }


def collective_and_sweep(Xd, W, reps=3):
    """The collective parallel form (Sec. 3.6, third scheme) on the medium
    workload, 8 workers x 7 rounds, checked against the oracle's stored
    result; and the sample-size rule of thumb (Sec. 5) from s = 5,000 with 50
    samples per size."""
    from paper_2204_07485_amd import bigmeans
    import torch
    with open(os.path.join(ROOT, "tests", "golden", "medium_collective.json")) as fh:
        gold = json.load(fh)
    kw = dict(max_iter=300, tol=1e-4, stop_rule=bigmeans.BM_STOP_REL_OBJ, n_local_trials=3)
    bigmeans.bigmeans_fit_collective(Xd, W.k, W.s, gold["workers"], gold["rounds"], W.seed, **kw)
    times, res = [], None
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = bigmeans.bigmeans_fit_collective(Xd, W.k, W.s, gold["workers"], gold["rounds"],
                                               W.seed, **kw)
        times.append((time.perf_counter() - t0) * 1e3)
    rel = abs(res["sse"] - gold["sse"]) / gold["sse"]
    ms = statistics.median(times)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sw = bigmeans.sample_size_sweep(Xd, W.k, 5_000, W.n, W.n_samples, W.seed, **kw)
    sweep_ms = (time.perf_counter() - t0) * 1e3
    return {
        "collective": {"workload": f"medium, {gold['workers']} workers x {gold['rounds']} rounds",
                       "ms": ms, "sse": res["sse"], "oracle_sse": gold["sse"],
                       "sse_rel_err": rel, "time_to_oracle_sse_ms": ms if rel <= 1e-6 else None,
                       "lloyd_iters": res["stats"]["lloyd_iters"],
                       "samples": res["stats"]["samples"]},
        "sample_size_sweep": {"workload": "medium, s = 5,000 doubling, 50 samples per size",
                              "ms": sweep_ms, "s_best": sw["s_best"], "sse": sw["sse"],
                              "tried": sw["tried"]},
    }


def final_passes(Xmed, gold, reps=5):
    """The full-data assignment pass (Alg. 1 last step) timed alone with HIP
    events, with the last-level cache flushed before each launch: the medium
    workload at its fitted centroids, and the batched workload's 10,000,000 x
    68 data (2.72 GB) at k = 50 (C = 50 of its rows)."""
    import numpy as np
    import torch

    from paper_2204_07485_amd import bigmeans, synth
    flush = torch.zeros(1 << 27, dtype=torch.float32, device="cuda:0")  # 512 MB
    res = {}
    Cm = np.array([[np.nan if v is None else v for v in row] for row in gold["C"]], np.float32)
    degm = np.array(gold["deg"], np.uint8)
    cases = [("medium_1Mx16_k25", Xmed, torch.from_numpy(Cm).cuda(), degm)]
    Xw = torch.from_numpy(synth.make_wide()).to("cuda:0")
    rows = np.random.default_rng(3).choice(Xw.shape[0], 50, replace=False)
    cases.append(("wide_10Mx68_k50", Xw, Xw[torch.from_numpy(rows).cuda()].contiguous(),
                  np.zeros(50, np.uint8)))
    for name, X, C, deg in cases:
        n, d = X.shape
        k = C.shape[0]
        vals = []
        for _ in range(reps):
            flush_mall(flush)
            bigmeans.kmeans_assign(X, C, deg)
            vals.append(bigmeans.last_assign_ms())
        warm = []
        for _ in range(reps):
            bigmeans.kmeans_assign(X, C, deg)
            warm.append(bigmeans.last_assign_ms())
        ms = statistics.median(vals)
        algo = n * d * 4 + n * 4
        # k d >= 256 (and d, k >= 8) runs on the matrix cores (same labels)
        mfma = d >= 8 and k >= 8 and k * d >= 256
        kernel = (f"assign_mfma32_kernel<{ {16: 1, 68: 5, 128: 8}[d] },true>" if mfma
                  else f"assign_kernel<{ {16: 16, 68: 72}[d] },f32>")
        res[name] = {"kernel": kernel, "ms_cold": ms,
                     "ms_warm": statistics.median(warm), "algorithmic_bytes": algo,
                     "gbs_cold": algo / (ms * 1e-3) / 1e9, "hbm_frac_cold": algo / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "tflops_cold": 2 * n * k * d / (ms * 1e-3) / 1e12}
        if mfma:  # issued matrix work: k padded to 16-row tiles, d to 16-column chunks
            kp, dp = 16 * -(-k // 16), 16 * {16: 1, 68: 5, 128: 8}[d]
            res[name]["mfma_tflops_cold"] = 2 * n * kp * dp / (ms * 1e-3) / 1e12
            res[name]["mfma_frac_cold"] = res[name]["mfma_tflops_cold"] / FP32_MFMA_PEAK_TFLOPS
    del Xw, flush
    torch.cuda.empty_cache()
    return res


def batched_solves(n_seq=16):
    """The batched workload: 10,000,000 x 68 FP32 (50 components, diagonal
    variances U[0.2, 3], Dirichlet weights, seed 3); 256 solves with
    s ~ U{5,000..100,000} and k cycling through (5, 10, 25, 50), each started
    like a Big-means run's first sample (its sample, rows and K-means++
    centres); then K-means on all of them at once, one graph launch per round,
    against the first n_seq solves run one after another."""
    import numpy as np
    import torch

    from paper_2204_07485_amd import bigmeans, synth
    X = torch.from_numpy(synth.make_wide()).to("cuda:0")
    solves = synth.wide_solves()
    P, s, k, C, deg = bigmeans.prepare_batch(X, solves)
    del X
    kw = dict(max_iter=300, tol=1e-4, stop_rule=bigmeans.BM_STOP_REL_OBJ)
    bigmeans.kmeans_lloyd_batched(P, s, k, C.clone(), deg, want_labels=False, **kw)  # tunes tiles
    Cr = C.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dg, _, f, passes, info = bigmeans.kmeans_lloyd_batched(P, s, k, Cr, deg, want_labels=False, **kw)
    wall = (time.perf_counter() - t0) * 1e3
    d = P.shape[1]
    rows_passes = float((passes.astype(np.float64) * s).sum())
    dev_ms = float(sum(info["round_ms"]))
    r0 = np.concatenate([[0], np.cumsum(s)])
    c0 = np.concatenate([[0], np.cumsum(k)])
    t1 = time.perf_counter()
    seq_rows = 0.0
    for j in range(n_seq):
        Cj = C[c0[j]:c0[j + 1]].clone()
        _, _, _, sp = bigmeans.kmeans_lloyd(P[r0[j]:r0[j + 1]], Cj, deg[c0[j]:c0[j + 1]], **kw)
        seq_rows += sp * s[j]
    seq_ms = (time.perf_counter() - t1) * 1e3
    # first round: every solve active, the full sample set streamed once;
    # algorithmic bytes count the 68 stored columns (the kernel reads rows
    # zero-padded to 72 columns, 6 % more)
    first_bytes = float(s.sum()) * d * 4
    first_ms = info["round_ms"][0]
    gbs = first_bytes / (first_ms * 1e-3) / 1e9
    return {
        "workload": "batched: 10,000,000 x 68 FP32 (50 components), 256 solves, s ~ U{5k..100k}, "
                    "k in (5,10,25,50), relative-objective stop 1e-4 / 300 rounds",
        "rows": int(s.sum()), "rounds": info["rounds"], "tile_rows": info["tile_rows"],
        "ms_wall": wall, "ms_device_rounds": dev_ms,
        "rows_x_passes_per_s": rows_passes / (wall * 1e-3),
        "sequential_rows_x_passes_per_s": seq_rows / (seq_ms * 1e-3),
        "speedup_vs_sequential": (rows_passes / wall) / (seq_rows / seq_ms),
        # labels from the matrix cores (kmax d >= 256): issued matrix work counts
        # k rounded up to 16-row tiles and 68 columns to five 16-column chunks
        "roofline_first_round": {"bound": "hbm", "kernel": "batch_assign_mfma32_kernel<5,true>",
                                 "achieved_gbs": gbs, "peak_gbs": HBM_PEAK_GBS,
                                 "algorithmic_bytes": first_bytes,
                                 "padded_bytes_read": float(s.sum()) * 72 * 4,
                                 "hbm_frac": gbs / HBM_PEAK_GBS, "ms": first_ms,
                                 "tflops": float((s * k).sum()) * 68 * 2 / (first_ms * 1e-3) / 1e12,
                                 "mfma_tflops": float((s * (16 * -(-k // 16))).sum()) * 80 * 2
                                                / (first_ms * 1e-3) / 1e12,
                                 "fp32_mfma_peak_tflops": FP32_MFMA_PEAK_TFLOPS},
    }


def serve_stream(n_jobs=200, slots=4, rate=200.0, seed=5):
    """The serving workload: Poisson arrivals (rate jobs/s) of jobs with
    n = floor(exp(U[ln 1e4, ln 1e6])), d from {2, 8, 16, 32, 68, 128}, k from
    U{2..50}, s = min(n, 50,000), 20 samples; each job's data is a k-component
    Gaussian mixture (means U[-10, 10]^d, sigma U[0.5, 2]) generated on the
    GPU from the job's seed before timing.  Jobs are submitted at their
    arrival times; latency = completion - arrival."""
    import numpy as np
    import torch

    from paper_2204_07485_amd import bigmeans, synth
    jobs = synth.serve_jobs(n_jobs, rate=rate, seed=seed)
    data = []
    for j in jobs:
        g = torch.Generator(device="cuda:0").manual_seed(j["seed"] % (2**63))
        means = torch.rand((j["k"], j["d"]), generator=g, device="cuda:0") * 20 - 10
        sig = torch.rand((j["k"], 1), generator=g, device="cuda:0") * 1.5 + 0.5
        comp = torch.randint(0, j["k"], (j["n"],), generator=g, device="cuda:0")
        X = means[comp] + sig[comp] * torch.randn((j["n"], j["d"]), generator=g, device="cuda:0")
        data.append(X.contiguous())
    torch.cuda.synchronize()
    kw = dict(max_iter=300, tol=1e-4, stop_rule=bigmeans.BM_STOP_REL_OBJ, n_local_trials=3)

    def run(mode, nslots, burst):
        with bigmeans.Server(slots=nslots, mode=mode) as srv:
            for j, X in list(zip(jobs, data))[:4]:  # warm-up
                srv.result(srv.submit(X, j["k"], j["s"], j["n_samples"], j["seed"], **kw))
            ids = []
            t0 = time.perf_counter()
            for j, X in zip(jobs, data):
                delay = t0 + j["arrival"] - time.perf_counter()
                if delay > 0 and not burst:
                    time.sleep(delay)
                ids.append(srv.submit(X, j["k"], j["s"], j["n_samples"], j["seed"], **kw))
            res = [srv.result(i) for i in ids]
            info = srv.info()
        sub = np.array([r["t_submit_ms"] for r in res])
        end = np.array([r["t_end_ms"] for r in res])
        lat = end - sub
        span_s = (end.max() - sub.min()) / 1e3
        return {
            "jobs": len(res), "jobs_per_s": len(res) / span_s,
            "latency_ms_p50": float(np.percentile(lat, 50)),
            "latency_ms_p99": float(np.percentile(lat, 99)),
            "service_ms_mean": float(np.mean(end - np.array([r["t_start_ms"] for r in res]))),
            "peak_scratch_mb": info["peak_reserved_bytes"] / 1e6, "failed": info["failed"]}

    out = {}
    # whole fits per slot (persistent solver) and continuous batching of the
    # jobs' Lloyd rounds; Poisson arrivals, then all jobs at once (capacity)
    for nslots in sorted({1, 2, slots}):
        out[f"fits_slots_{nslots}"] = run(bigmeans.BM_SERVE_FITS, nslots, False)
    for nslots in (8, 16):
        out[f"rounds_slots_{nslots}"] = run(bigmeans.BM_SERVE_ROUNDS, nslots, False)
    out["burst_fits_slots_1"] = run(bigmeans.BM_SERVE_FITS, 1, True)
    out["burst_rounds_slots_16"] = run(bigmeans.BM_SERVE_ROUNDS, 16, True)
    out["workload"] = (f"serving: {n_jobs} jobs, Poisson arrivals at {rate:g}/s, n log-uniform in "
                       "[1e4, 1e6], d in {2,8,16,32,68,128}, k in [2,50], s = min(n, 50,000), "
                       "20 samples, seed 5")
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU only (asked for {args.gpus}); "
              "multi-GPU sharding is not built", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2204_07485_amd import bigmeans, synth

    W = synth.MEDIUM
    with open(os.path.join(ROOT, "tests", "golden", "medium_fit.json")) as fh:
        gold = json.load(fh)
    X = synth.make_medium()
    Xd = torch.from_numpy(X).to("cuda:0")
    torch.cuda.synchronize()
    kw = dict(max_iter=300, tol=1e-4, stop_rule=bigmeans.BM_STOP_REL_OBJ, n_local_trials=3)

    def fit():
        return bigmeans.bigmeans_fit(Xd, W.k, W.s, W.n_samples, W.seed, **kw)

    for i in range(args.warmup):
        fit()
        print(f"warmup {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)

    torch.cuda.synchronize()
    wall = []
    results = []
    t_start = time.perf_counter()
    for i in range(args.steps):
        t0 = time.perf_counter()
        r = fit()
        wall.append((time.perf_counter() - t0) * 1e3)
        results.append(r)
    torch.cuda.synchronize()
    total_ms = (time.perf_counter() - t_start) * 1e3
    ms_per_step = total_ms / args.steps
    print(f"timed {args.steps} fits: {ms_per_step:.3f} ms/fit", file=sys.stderr, flush=True)

    rel = [abs(r["sse"] - gold["sse"]) / gold["sse"] for r in results]
    matched = max(rel) <= 1e-6
    st = results[-1]["stats"]
    solver_ms = statistics.mean(r["stats"]["ms_solver"] for r in results)
    final_ms = statistics.mean(r["stats"]["ms_final"] for r in results)

    # algorithmic bytes of the solver kernel per launch: every Lloyd pass reads
    # the sample (s x d FP32) once; every sample gathers s rows of X and writes
    # them to the sample buffer
    s, d, n, k = W.s, W.d, W.n, W.k
    passes = st["lloyd_iters"]
    solver_bytes = passes * s * d * 4 + W.n_samples * s * d * 4 * 2
    solver_flops = passes * s * k * d * 2
    final_bytes = n * d * 4 + n * 4
    final_flops = n * k * d * 2
    achieved = solver_bytes / (solver_ms * 1e-3) / 1e9
    final_gbs = final_bytes / (final_ms * 1e-3) / 1e9
    traffic_solver, traffic_final = measured_traffic()

    line = {
        "metric": "Big-means time-to-oracle-SSE; assign TFLOP/s & HBM GB/s; p50/p99 job latency",
        "value": ms_per_step if matched else None,
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "medium: 1,000,000 x 16 FP32 Gaussian mixture (25 components), "
                               "k=25, s=40,000, 50 samples, seed 2, stop: relative objective "
                               "decrease <= 1e-4 or 300 rounds, 3 K-means++ candidates, "
                               "then full-data assign + SSE",
                   "n": n, "d": d, "k": k, "s": s, "n_samples": W.n_samples,
                   "grid": st["grid"]},
        "oracle_sse_match": matched,
        "sse": results[-1]["sse"],
        "oracle_sse": gold["sse"],
        "sse_rel_err_max": max(rel),
        "fit_ms_p50": float(np.percentile(wall, 50)),
        "fit_ms_p99": float(np.percentile(wall, 99)),
        "roofline": {"bound": "hbm", "kernel": "sample loop: presample_collect/select/emit<16> + solver_kernel<16>",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic_solver,
                     "ms_per_launch": solver_ms, "algorithmic_bytes": solver_bytes,
                     "tflops": solver_flops / (solver_ms * 1e-3) / 1e12},
        "roofline_final_pass": {"bound": "hbm", "kernel": "assign_mfma32_kernel<1,true>",
                                "achieved": final_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                "frac": final_gbs / HBM_PEAK_GBS, "traffic": traffic_final,
                                "ms_per_launch": final_ms,
                                "algorithmic_bytes": final_bytes,
                                "tflops": final_flops / (final_ms * 1e-3) / 1e12},
        "stats": st,
    }
    if args.copy_calibration:
        src = torch.empty(1 << 28, dtype=torch.float32, device="cuda:0").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if not args.no_extras:
        print("collective mode and sample-size sweep ...", file=sys.stderr, flush=True)
        line.update(collective_and_sweep(Xd, W))
    if not args.no_final:
        print("final passes (cache flushed) ...", file=sys.stderr, flush=True)
        line["final_pass"] = final_passes(Xd, gold)
    if not args.no_mixed:
        print("mixed precision: BF16 workload ...", file=sys.stderr, flush=True)
        line["mixed_precision"] = mixed_precision()
    if not args.no_batch:
        print("batched solves ...", file=sys.stderr, flush=True)
        line["batched"] = batched_solves()
    if not args.no_serve:
        print("serving stream ...", file=sys.stderr, flush=True)
        line["serving"] = serve_stream()
    if not args.no_cpu_baseline:
        print("cpu baseline (oracle, all host cores) ...", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(X, W)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
