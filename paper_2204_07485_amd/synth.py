"""Seeded synthetic inputs shaped like the paper's workloads.

The paper evaluates on public datasets (its Tables 1-2) that are not shipped
here; seeded Gaussian mixtures with the same kinds of shapes stand in for them.
This module holds only input generation (numpy ``default_rng``), none of the
clustering arithmetic, and serves both the GPU path and the CPU oracle: X is
generated once and handed to both unchanged.

Workloads (n points x d features, k clusters, sample size s, T samples):
  small   20,000 x 8, 10 isotropic components (sigma 1, equal weights),
          k=10, s=2,000, T=20
  medium  1,000,000 x 16, 25 components (sigma_c ~ U[0.5, 2], Dirichlet(1)
          weights), k=25, s=40,000, T=50
  wide    10,000,000 x 68, 50 components, per-dimension variances
          ~ U[0.2, 3], Dirichlet(1) weights (batched solves)
  bf16    5,000,000 x 128 stored as BF16, 100 components (sigma_c ~ U[0.5, 2])
          plus 10 % uniform outliers, k=100, s=200,000, T=30
  serve   a Poisson stream of jobs with n ~ logU[1e4, 1e6],
          d in {2, 8, 16, 32, 68, 128}, k ~ U{2..50}
Component means are ~ U[-10, 10]^d in every workload.
"""
from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Workload:
    name: str
    n: int
    d: int
    k: int
    s: int
    n_samples: int
    seed: int
    max_iter: int = 100
    tol: float = 1e-4


SMALL = Workload("small", 20_000, 8, 10, 2_000, 20, seed=1)
MEDIUM = Workload("medium", 1_000_000, 16, 25, 40_000, 50, seed=2)
BF16 = Workload("bf16", 5_000_000, 128, 100, 200_000, 30, seed=4)


def gaussian_mixture(n, d, n_comp, seed, sigma=None, sigma_range=None, var_range=None,
                     weights="equal", outlier_frac=0.0, chunk=1 << 20):
    """Return (X float32 (n, d), component id int32 (n,)).

    Exactly one of sigma (isotropic, shared), sigma_range (isotropic per
    component, U[lo, hi]) or var_range (diagonal variances per component and
    dimension, U[lo, hi]) sets the spread.  Outliers (a fraction of the rows,
    at random positions, component id -1) are uniform over the box spanned by
    the means widened by 3 on every side.
    """
    rng = np.random.default_rng(seed)
    means = rng.uniform(-10.0, 10.0, size=(n_comp, d))
    if sigma is not None:
        scale = np.full((n_comp, d), float(sigma))
    elif sigma_range is not None:
        scale = np.repeat(rng.uniform(*sigma_range, size=(n_comp, 1)), d, axis=1)
    elif var_range is not None:
        scale = np.sqrt(rng.uniform(*var_range, size=(n_comp, d)))
    else:
        raise ValueError("one of sigma, sigma_range, var_range is required")
    if weights == "equal":
        w = np.full(n_comp, 1.0 / n_comp)
    elif weights == "dirichlet":
        w = rng.dirichlet(np.ones(n_comp))
    else:
        raise ValueError(weights)
    comp = rng.choice(n_comp, size=n, p=w).astype(np.int32)
    means32 = means.astype(np.float32)
    scale32 = scale.astype(np.float32)
    X = np.empty((n, d), dtype=np.float32)
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        z = rng.standard_normal((hi - lo, d), dtype=np.float32)
        c = comp[lo:hi]
        X[lo:hi] = means32[c] + scale32[c] * z
    if outlier_frac > 0.0:
        n_out = int(round(outlier_frac * n))
        rows = rng.choice(n, size=n_out, replace=False)
        lo_b = means.min() - 3.0
        hi_b = means.max() + 3.0
        X[rows] = rng.uniform(lo_b, hi_b, size=(n_out, d)).astype(np.float32)
        comp[rows] = -1
    return X, comp


def to_bf16_bits(X):
    """Round float32 to bfloat16 (round to nearest even); returns uint16 bits."""
    u = np.ascontiguousarray(X, dtype=np.float32).view(np.uint32)
    bias = np.uint32(0x7FFF) + ((u >> np.uint32(16)) & np.uint32(1))
    return ((u + bias) >> np.uint32(16)).astype(np.uint16)


def bf16_bits_to_f32(H):
    return (np.ascontiguousarray(H, dtype=np.uint16).astype(np.uint32) << np.uint32(16)).view(np.float32)


def make_small():
    return gaussian_mixture(SMALL.n, SMALL.d, 10, SMALL.seed, sigma=1.0)[0]


def make_medium():
    return gaussian_mixture(MEDIUM.n, MEDIUM.d, 25, MEDIUM.seed, sigma_range=(0.5, 2.0),
                            weights="dirichlet")[0]


def make_wide(n=10_000_000):
    return gaussian_mixture(n, 68, 50, 3, var_range=(0.2, 3.0), weights="dirichlet")[0]


def make_bf16(n=BF16.n):
    X, _ = gaussian_mixture(n, BF16.d, 100, BF16.seed, sigma_range=(0.5, 2.0),
                            outlier_frac=0.10)
    return to_bf16_bits(X)


def wide_solves(n_solves=256, seed=3):
    """Per-solve (s, k, seed) for the batched workload: s ~ U{5,000..100,000},
    k cycling through (5, 10, 25, 50)."""
    rng = np.random.default_rng(seed + 1000)
    s = rng.integers(5_000, 100_001, size=n_solves)
    ks = np.array([(5, 10, 25, 50)[i % 4] for i in range(n_solves)])
    seeds = rng.integers(1, 2**63 - 1, size=n_solves, dtype=np.int64)
    return [(int(s[i]), int(ks[i]), int(seeds[i])) for i in range(n_solves)]


def serve_jobs(n_jobs, rate=200.0, seed=5, n_range=(1e4, 1e6), s_cap=50_000):
    """Poisson arrivals of clustering jobs: list of dicts with arrival time (s),
    n, d, k, s, seed (the job's data is made by serve_job_data)."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=n_jobs)
    t = np.cumsum(gaps) - gaps[0]
    jobs = []
    for j in range(n_jobs):
        n = int(np.floor(np.exp(rng.uniform(np.log(n_range[0]), np.log(n_range[1])))))
        d = int(rng.choice([2, 8, 16, 32, 68, 128]))
        k = int(rng.integers(2, 51))
        jobs.append({"id": j, "arrival": float(t[j]), "n": n, "d": d, "k": k,
                     "s": min(n, s_cap), "n_samples": 20,
                     "seed": int(rng.integers(1, 2**62))})
    return jobs


def serve_job_data(job):
    X, _ = gaussian_mixture(job["n"], job["d"], job["k"], job["seed"], sigma_range=(0.5, 2.0))
    return X
