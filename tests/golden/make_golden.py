"""Write the stored oracle results used by the GPU tests and the benchmark.

Calls only the CPU oracle (oracle/) on the seeded synthetic inputs of
paper_2204_07485_amd.synth; nothing here comes from the GPU path.

    python tests/golden/make_golden.py [medium] [bf16]

medium_fit.json (about half a minute): Big-means on the medium workload
(1,000,000 x 16, 25 components, k=25, s=40,000, 50 samples, seed 2) with the
paper's stop rule (relative objective decrease <= 1e-4 or 300 rounds, Sec. 5)
and three K-means++ candidates (Sec. 5), followed by the final assignment.

medium_collective.json: the collective parallel form (Sec. 3.6, third scheme)
on the medium workload: 8 workers x 7 rounds (56 samples), same stop rule and
seeding, followed by the final assignment (threaded oracle build).

bf16_fit.json (minutes on all host cores; the threaded oracle build,
whose results are bit-identical to the single-threaded one): the same on the
BF16 workload (5,000,000 x 128 stored as BF16, 100 components plus 10 %
uniform outliers, k=100, s=200,000, 30 samples, seed 4); the oracle reads the
BF16 values widened exactly.
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_2204_07485_amd import synth  # noqa: E402


def medium():
    W = synth.MEDIUM
    X = synth.make_medium()
    t0 = time.time()
    r = oracle.bigmeans_fit(X, W.k, W.s, W.n_samples, W.seed, max_iter=300, tol=1e-4,
                            stop_rule=oracle.ORC_STOP_REL_OBJ, n_local_trials=3,
                            want_labels=True)
    secs = time.time() - t0
    out = {
        "workload": "medium: 1,000,000 x 16, k=25, s=40,000, 50 samples, seed 2, "
                    "stop: relative objective decrease <= 1e-4 or 300 rounds",
        "sse": r["sse"], "f_opt": r["f_opt"], "sample_f": r["sample_f"].tolist(),
        "deg": r["deg"].tolist(),
        "C": np.where(np.isnan(r["C"]), None, r["C"]).tolist(),
        "label_counts": np.bincount(r["labels"], minlength=W.k).tolist(),
        "stats": r["stats"], "oracle_seconds_single_thread": secs,
    }
    with open(os.path.join(HERE, "medium_fit.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print(f"medium: sse={r['sse']!r} f_opt={r['f_opt']!r} in {secs:.1f}s", flush=True)


def bf16():
    W = synth.BF16
    H = synth.make_bf16()
    t0 = time.time()
    with oracle.threaded():
        threads = oracle.threads()
        r = oracle.bigmeans_fit(H, W.k, W.s, W.n_samples, W.seed, max_iter=300, tol=1e-4,
                                stop_rule=oracle.ORC_STOP_REL_OBJ, n_local_trials=3,
                                want_labels=True, x_dtype=oracle.ORC_BF16)
    secs = time.time() - t0
    out = {
        "workload": "bf16: 5,000,000 x 128 BF16, 100 components + 10% uniform outliers, k=100, "
                    "s=200,000, 30 samples, seed 4, stop: relative objective decrease <= 1e-4 "
                    "or 300 rounds",
        "sse": r["sse"], "f_opt": r["f_opt"], "sample_f": r["sample_f"].tolist(),
        "deg": r["deg"].tolist(),
        "C": np.where(np.isnan(r["C"]), None, r["C"]).tolist(),
        "label_counts": np.bincount(r["labels"][r["labels"] >= 0], minlength=W.k).tolist(),
        "stats": r["stats"], "oracle_seconds": secs, "oracle_threads": threads,
    }
    with open(os.path.join(HERE, "bf16_fit.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print(f"bf16: sse={r['sse']!r} f_opt={r['f_opt']!r} in {secs:.1f}s on {threads} threads",
          flush=True)


def collective():
    W = synth.MEDIUM
    X = synth.make_medium()
    workers, rounds = 8, 7
    t0 = time.time()
    with oracle.threaded():
        r = oracle.bigmeans_collective(X, W.k, W.s, workers, rounds, W.seed, max_iter=300,
                                       tol=1e-4, stop_rule=oracle.ORC_STOP_REL_OBJ,
                                       n_local_trials=3, want_labels=True)
    secs = time.time() - t0
    out = {
        "workload": "medium, collective: 1,000,000 x 16, k=25, s=40,000, 8 workers x 7 rounds, "
                    "seed 2, stop: relative objective decrease <= 1e-4 or 300 rounds",
        "workers": workers, "rounds": rounds,
        "sse": r["sse"], "f_opt": r["f_opt"], "worker_f": r["worker_f"].tolist(),
        "deg": r["deg"].tolist(),
        "C": np.where(np.isnan(r["C"]), None, r["C"]).tolist(),
        "label_counts": np.bincount(r["labels"], minlength=W.k).tolist(),
        "stats": r["stats"], "oracle_seconds": secs,
    }
    with open(os.path.join(HERE, "medium_collective.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print(f"collective: sse={r['sse']!r} f_opt={r['f_opt']!r} in {secs:.1f}s", flush=True)


if __name__ == "__main__":
    targets = sys.argv[1:] or ["medium"]
    for name in targets:
        {"medium": medium, "bf16": bf16, "collective": collective}[name]()
