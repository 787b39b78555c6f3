"""Pins for the oracle's random stream (CPU).

Philox4x32-10 is checked against rocRAND's independent implementation of the
same generator; the derived draws (unit double, bounded integer, sample keys)
against their arithmetic definitions and distribution laws.
"""
import os
import subprocess

import numpy as np
import pytest
from scipy import stats

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
REF_SRC = os.path.join(HERE, "rocrand_philox_ref.cpp")
REF_BIN = os.path.join(HERE, "_build", "rocrand_philox_ref")


def _rocrand_ref():
    os.makedirs(os.path.dirname(REF_BIN), exist_ok=True)
    if not os.path.exists(REF_BIN) or os.path.getmtime(REF_BIN) < os.path.getmtime(REF_SRC):
        subprocess.run(["hipcc", "-O1", "-std=c++17", REF_SRC, "-o", REF_BIN], check=True)
    return REF_BIN


def _cases(n, seed=123):
    rng = np.random.default_rng(seed)
    seeds = rng.integers(0, 2**64, size=n, dtype=np.uint64)
    ctrs = rng.integers(0, 2**32, size=(n, 4), dtype=np.uint64)
    edge_seeds = np.array([0, 1, 2**32 - 1, 2**32, 2**64 - 1], dtype=np.uint64)
    edge_ctrs = np.array([[0, 0, 0, 0], [1, 0, 0, 0], [0, 0, 0, 1],
                          [2**32 - 1] * 4, [5, 0, 7, 1]], dtype=np.uint64)
    return np.concatenate([edge_seeds, seeds]), np.concatenate([edge_ctrs, ctrs])


def test_philox_matches_rocrand():
    exe = _rocrand_ref()
    seeds, ctrs = _cases(5000)
    lines = "\n".join(f"{int(s)} {int(c[0])} {int(c[1])} {int(c[2])} {int(c[3])}"
                      for s, c in zip(seeds, ctrs)) + "\n"
    out = subprocess.run([exe], input=lines, capture_output=True, text=True, check=True).stdout
    ref = np.array([[int(v) for v in ln.split()] for ln in out.strip().splitlines()],
                   dtype=np.uint64)
    assert ref.shape == (len(seeds), 4)
    for s, c, r in zip(seeds, ctrs, ref):
        key = [int(s) & 0xFFFFFFFF, int(s) >> 32]
        got = oracle.philox([int(v) for v in c], key)
        assert [int(v) for v in got] == [int(v) for v in r], (int(s), c)


def test_seed_word_layout():
    # draw q of sample t: counter (lo32(q), hi32(q), t, 1), word = out0 << 32 | out1
    for seed, t, q in [(7, 0, 0), (2**40 + 3, 5, 2**33 + 9), (1, 2**31, 17)]:
        out = oracle.philox([q & 0xFFFFFFFF, q >> 32, t, 1], [seed & 0xFFFFFFFF, seed >> 32])
        assert oracle.seed_word(seed, t, q) == (int(out[0]) << 32) | int(out[1])


def test_sample_key_layout():
    # point i of sample t: block i//2 with counter (lo32, hi32, t, 0); even i
    # takes words 0-1, odd i words 2-3
    for seed, t, i in [(3, 0, 0), (3, 0, 1), (99, 4, 2**32 + 5), (99, 4, 2**32 + 4)]:
        b = i >> 1
        out = oracle.philox([b & 0xFFFFFFFF, b >> 32, t, 0], [seed & 0xFFFFFFFF, seed >> 32])
        want = ((int(out[0]) << 32) | int(out[1])) if i % 2 == 0 else \
               ((int(out[2]) << 32) | int(out[3]))
        assert oracle.sample_key(seed, t, i) == want


def test_keys_look_uniform():
    keys = np.array([oracle.sample_key(11, 0, i) for i in range(20000)], dtype=np.uint64)
    top = (keys >> np.uint64(60)).astype(np.int64)   # 16 bins
    counts = np.bincount(top, minlength=16)
    assert stats.chisquare(counts).pvalue > 1e-4
    assert len(np.unique(keys)) == len(keys)
